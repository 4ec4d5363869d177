"""GPU parity of joints (sec. 5.3: material points of two bodies, or of a
body and the world, made to coincide; a hinge is two such joints on its
axis; stiff quadratic penalty) against the oracle: the joint terms inside a
Newton step's gradient and Hessian (diagonal and off-diagonal blocks, the
off-diagonal pattern with the joint pairs), Newton steps, 30 time steps of
a swinging five-link hinged chain, two chains as sub-scenes of one batch,
and one adjoint step."""
import numpy as np
import pytest

import oracle
import scenegen as sg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def abd():
    import paper_2201_10022_amd as abd
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return abd


@pytest.fixture(scope="module")
def ctx(abd):
    return abd.Context(0)


def _dev(a, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda:0")


def test_joint_pattern_and_newton_step(abd, ctx):
    S, P = sg.hinged_chain()
    P = dict(P, pcg_rtol=1e-14, max_pcg=20000)
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    B = oracle.Body(S)
    empty = np.zeros((0, 2), np.int32)
    keys = ctx.offdiag_pattern(sc, _dev(empty, torch.int32), _dev(empty, torch.int32)).cpu().numpy()
    np.testing.assert_array_equal(keys, oracle.off_keys(S, empty, empty))
    assert len(keys) == 4
    rng = np.random.default_rng(3)
    q = S["q0"] + 1e-4 * rng.normal(size=S["q0"].shape)
    qt = oracle.q_tilde(S, q, S["qd0"], P)
    qn_ref, conv, info = oracle.newton_iteration(S, B, q, qt, P)
    assert not conv
    qg = _dev(q)
    st = ctx.newton_step(sc, P, qg, _dev(qt))
    ref = qn_ref - q
    err = np.abs(qg.cpu().numpy() - q - ref).max() / np.abs(ref).max()
    assert err <= 1e-8, err
    assert st["alpha"] == pytest.approx(info["alpha"], rel=1e-9)


def test_hinged_chain_trajectory(abd, ctx):
    S, P = sg.hinged_chain()
    P = dict(P, pcg_rtol=1e-13, max_pcg=20000)
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    B = oracle.Body(S)
    q, qd = S["q0"].copy(), S["qd0"].copy()
    qg, qdg = _dev(q), _dev(qd)
    for step in range(30):
        q, qd, _ = oracle.time_step(S, B, q, qd, P)
        st = ctx.time_step(sc, P, qg, qdg)
        assert st["converged"] == 1
        np.testing.assert_allclose(qg.cpu().numpy(), q, rtol=0, atol=1e-6)
    # the chain swung (the tip moved by more than 10 cm) and its hinges held
    assert np.abs(q[-1, :3] - S["q0"][-1, :3]).max() > 0.1
    for (a, b), (pa, pb) in zip(S["joint_body"], S["joint_point"]):
        xa = q[a, :3] + q[a, 3:].reshape(3, 3) @ pa
        xb = pb if b < 0 else q[b, :3] + q[b, 3:].reshape(3, 3) @ pb
        assert np.linalg.norm(xa - xb) < 1e-4


def test_two_chains_as_sub_scenes(abd, ctx):
    # two hinged chains in one scene and as two sub-scenes of a batch: the
    # batch's time steps equal the single scene's per sub-scene
    S, P = sg.hinged_chain(n_chains=2)
    P = dict(P, pcg_rtol=1e-13, max_pcg=20000)
    Sb = dict(S)
    nb = len(S["q0"])
    Sb["body_scene"] = (np.arange(nb) >= nb // 2).astype(np.int32)
    Sb["scene_body_off"] = np.array([0, nb // 2, nb], np.int32)
    sc, scb = abd.Scene(S), abd.Scene(Sb)
    ctx.body_mass(sc)
    ctx.body_mass(scb)
    q, qd = _dev(S["q0"]), _dev(S["qd0"])
    qb, qdb = _dev(S["q0"]), _dev(S["qd0"])
    for _ in range(10):
        ctx.time_step(sc, P, q, qd)
        ctx.time_step(scb, P, qb, qdb)
    np.testing.assert_allclose(qb.cpu().numpy(), q.cpu().numpy(), rtol=0, atol=1e-6)


def test_adjoint_step_with_joints(abd, ctx):
    S, P = sg.hinged_chain(n_links=3)
    P = dict(P, newton_tol=1e-7)
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    B = oracle.Body(S)
    q, qd = S["q0"].copy(), S["qd0"].copy()
    for _ in range(3):
        q, qd, _ = oracle.time_step(S, B, q, qd, P)
    q_next, _, _ = oracle.time_step(S, B, q, qd, P)
    rng = np.random.default_rng(7)
    qbar, qdbar = rng.normal(size=q.shape), rng.normal(size=q.shape)
    rq, rqd = oracle.adjoint_step(S, B, q, qd, q_next, qbar, qdbar, P, None)
    gq, gqd, its = ctx.adjoint_step(sc, P, _dev(q), _dev(qd), _dev(q_next), _dev(qbar), _dev(qdbar), rtol=1e-13)
    np.testing.assert_allclose(gq.cpu().numpy(), rq, rtol=0, atol=1e-8 * np.abs(rq).max())
    np.testing.assert_allclose(gqd.cpu().numpy(), rqd, rtol=0, atol=1e-8 * np.abs(rqd).max())

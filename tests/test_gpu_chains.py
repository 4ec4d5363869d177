"""GPU parity on the dense-contact chain workload (64 interlocked links,
640,000 vertices, 1.28 M triangles; dt 5e-3, dhat 5e-4), the stand-in for
the paper's chain-net scenes (sec. 5, Tab. tab:time).

At full size: a contact state built from positions only (every upright
link moved 1.95 mm along its chain towards the next flat link, chains moved
1.95 mm closer together, so interlocked and side-by-side neighbours sit
5e-5 apart before the vertex noise): static candidates bit-exact, the
barrier gradient and projected Hessian blocks within 1e-10, and the swept
candidates and CCD bounds of the links' initial velocities over one step.
On a sub-chain (2 chains x 3 links, 100 x 25 mesh): Newton steps within
1e-8 of the oracle's (one cut by CCD, one with active contacts), and ten
time steps (links colliding at their initial velocities) within 1e-6 of
the oracle's trajectory."""
import numpy as np
import pytest

import oracle
import scenegen as sg
from parity_scales import abs_scale

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


def _sorted(a):
    a = np.asarray(a, dtype=np.int64).reshape(-1, 2)
    return a[np.lexsort((a[:, 1], a[:, 0]))] if len(a) else a


def test_chains_full_size_candidates_barrier_ccd(abd, ctx):
    S, P = sg.torus_chains()
    assert len(S["xbar"]) == 640000 and len(S["tris"]) == 1280000
    sc = abd.Scene(S)
    q = sg.torus_chains_contact(S, 8)
    x = oracle.vertex_map(S, q)
    xg = _dev(x)
    pt, ee = oracle.candidates(S, x, None, P["dhat"])
    gpt, gee = ctx.candidates(sc, xg, None, P["dhat"])
    np.testing.assert_array_equal(_sorted(gpt.cpu().numpy()), pt)
    np.testing.assert_array_equal(_sorted(gee.cpu().numpy()), ee)
    keys = oracle.off_keys(S, pt, ee)
    np.testing.assert_array_equal(ctx.offdiag_pattern(sc, gpt, gee).cpu().numpy(), keys)
    assert len(keys) >= 16
    r, gs, Ds, Os = abs_scale(S, x, pt, ee, P, keys)
    assert r["n_active"] >= 20
    e, g, D, O = ctx.barrier_grad_hess(sc, P, xg, _dev(pt, torch.int32), _dev(ee, torch.int32),
                                       _dev(keys, torch.int32))
    tol = 1e-10
    assert abs(e.item() - r["energy"]) <= tol * abs(r["energy"])

    def worst(a, b, s):
        return float(np.max(np.abs(a - b) / np.maximum(s, 1e-300)))

    errs = dict(g=worst(g.cpu().numpy(), r["grad"], gs), D=worst(D.cpu().numpy(), r["diag"], Ds),
                O=worst(O.cpu().numpy(), r["off"], Os))
    assert max(errs.values()) <= tol, errs
    # one step of the initial velocities: swept candidates and CCD
    x1 = oracle.vertex_map(S, q + P["dt"] * S["qd0"])
    spt, see = oracle.candidates(S, x, x1, P["dhat"])
    gspt, gsee = ctx.candidates(sc, xg, _dev(x1), P["dhat"])
    np.testing.assert_array_equal(_sorted(gspt.cpu().numpy()), spt)
    np.testing.assert_array_equal(_sorted(gsee.cpu().numpy()), see)
    assert len(spt) + len(see) > 10000
    tp, te, alpha = ctx.ccd_max_step(sc, P, xg, _dev(x1 - x), _dev(spt, torch.int32), _dev(see, torch.int32))
    otp, ote, oalpha = oracle.ccd(S, x, x1 - x, spt, see, P)
    for t, ot in ((tp.cpu().numpy(), otp), (te.cpu().numpy(), ote)):
        assert np.all(t <= ot * (1 + 1e-9))
        assert np.all(t >= 0.99 * ot)
    assert oalpha < 1.0
    assert oalpha * 0.99 <= alpha.item() <= oalpha * (1 + 1e-9)


def test_subchain_newton_steps(abd, ctx):
    # 2 chains x 3 links (100 x 25 mesh): the oracle's own two time steps
    # bring the middle links within one step of their neighbours; at step
    # 3 the first Newton iteration is cut by CCD and the second has active
    # contacts: both against the oracle's iterations from the same state
    S, P = sg.torus_chains(n_chains=2, n_links=3, n_major=100, n_minor=25)
    P = dict(P, newton_tol=1e-5, pcg_rtol=1e-14, max_pcg=20000)
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    B = oracle.Body(S)
    q, qd = S["q0"].copy(), S["qd0"].copy()
    for _ in range(2):
        q, qd, _ = oracle.time_step(S, B, q, qd, P)
    qt = oracle.q_tilde(S, q, qd, P)
    seen = dict(ccd_cut=False, active=False)
    for it in range(2):
        qn_ref, conv_ref, info = oracle.newton_iteration(S, B, q, qt, P)
        assert not conv_ref
        qg = _dev(q)
        st = ctx.newton_step(sc, P, qg, _dev(qt))
        assert st["n_active_pt"] + st["n_active_ee"] == info["n_active"]
        assert st["alpha"] == pytest.approx(info["alpha"], rel=1e-9)
        ref = qn_ref - q
        err = np.abs(qg.cpu().numpy() - q - ref).max() / np.abs(ref).max()
        assert err <= 1e-8, (it, err)
        seen["ccd_cut"] |= info["alpha"] < 0.9
        seen["active"] |= info["n_active"] > 0
        q = qn_ref
    assert seen["ccd_cut"] and seen["active"]


def test_subchain_trajectory(abd, ctx):
    # ten steps of a 2 x 3 sub-chain (links at 100 x 25 mesh resolution)
    # from the generator's state: the middle links hit their neighbours
    # within the first steps and keep colliding
    S, P = sg.torus_chains(n_chains=2, n_links=3, n_major=100, n_minor=25)
    P = dict(P, newton_tol=1e-5, pcg_rtol=1e-13, max_pcg=20000)
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    B = oracle.Body(S)
    q, qd = S["q0"].copy(), S["qd0"].copy()
    qg, qdg = _dev(q), _dev(qd)
    contact_steps = 0
    for step in range(10):
        log = []
        q, qd, its = oracle.time_step(S, B, q, qd, P, log=log)
        st = ctx.time_step(sc, P, qg, qdg)
        assert st["converged"] == 1
        np.testing.assert_allclose(qg.cpu().numpy(), q, rtol=0, atol=1e-6)
        contact_steps += max(l["n_active"] for l in log) > 0
    assert contact_steps >= 5

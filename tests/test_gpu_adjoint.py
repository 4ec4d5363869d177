"""GPU parity of the adjoint (reverse mode of the implicit-Euler step and of
checkpointed rollouts) against the CPU oracle's adjoint, which the CPU
suite pins by central differences.  Bars: one reverse step 1e-8 of the
largest entry (PCG at relative residual 1e-13 vs the oracle's direct
solve); rollout gradients 1e-5 relative (the two forward trajectories agree
to the Newton tolerance); checkpoint spacing changes nothing (bit-exact);
the autograd function returns the library's gradient unchanged."""
import math

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


def _cases():
    out = []
    S = sg.near_contact_cubes(4, n=4)
    P = sg.default_params(newton_tol=1e-7, max_newton=400)
    out.append(("cubes", S, P))
    S, P = sg.cube_on_slope(math.atan(0.75), 0.5, v0=1.0)
    out.append(("slope_friction", S, dict(P, newton_tol=1e-9, max_newton=400)))
    S = sg.near_contact_cubes(5, n=3)
    out.append(("cubes_friction", S, sg.default_params(newton_tol=1e-7, max_newton=400, mu=0.4)))
    return out


CASES = _cases()


@pytest.mark.parametrize("solver", ["cg_first", "minres"])
@pytest.mark.parametrize("name,S,P", CASES, ids=[c[0] for c in CASES])
def test_adjoint_step_parity(abd, ctx, name, S, P, solver, monkeypatch):
    # (the adjoint solve is CG with MINRES where CG fails; ABD_ADJ_MINRES=1
    # runs MINRES alone, so both solvers meet the oracle on every case)
    if solver == "minres":
        monkeypatch.setenv("ABD_ADJ_MINRES", "1")
    else:
        monkeypatch.delenv("ABD_ADJ_MINRES", raising=False)
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    B = oracle.Body(S)
    q, qd = S["q0"].copy(), S["qd0"].copy()
    free = S["body_fixed"] == 0
    if name != "slope_friction":
        qd[free, 1] -= 0.05
    for _ in range(3):  # a few steps so contacts are active
        q, qd, _ = oracle.time_step(S, B, q, qd, P)
    q_next, qd_next, _ = oracle.time_step(S, B, q, qd, P)
    rng = np.random.default_rng(3)
    qbar = rng.normal(size=q.shape) * free[:, None]
    qdbar = rng.normal(size=q.shape) * free[:, None]
    F = oracle.step_friction(S, q, P)
    rq, rqd = oracle.adjoint_step(S, B, q, qd, q_next, qbar, qdbar, P, F)
    gq, gqd, its = ctx.adjoint_step(sc, P, _dev(q), _dev(qd), _dev(q_next), _dev(qbar), _dev(qdbar), rtol=1e-13)
    assert its > 0
    np.testing.assert_allclose(gq.cpu().numpy(), rq, rtol=0, atol=1e-8 * np.abs(rq).max())
    np.testing.assert_allclose(gqd.cpu().numpy(), rqd, rtol=0, atol=1e-8 * np.abs(rqd).max())


def _loss_grad(S, q_T):
    b1 = int(np.flatnonzero(S["body_fixed"] == 0)[0])
    target = np.array([0.3, 0.4, -0.2])
    g = np.zeros_like(q_T)
    g[b1, :3] = 2 * (q_T[b1, :3] - target)
    return g


@pytest.mark.parametrize("name,S,P,n", [("three_cubes", *sg.three_cubes(), 20), ("slope_friction", *CASES[1][1:], 15)],
                         ids=["three_cubes", "slope_friction"])
def test_rollout_backward_matches_oracle(abd, ctx, name, S, P, n):
    P = dict(P, newton_tol=min(P["newton_tol"], 1e-7), max_newton=400, pcg_rtol=1e-13, max_pcg=20000)
    S = dict(S)
    if name == "three_cubes":
        S["qd0"] = S["qd0"].copy()
        S["qd0"][1:, 1] = -0.5
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    B = oracle.Body(S)
    states, _ = oracle.rollout(S, B, S["q0"], S["qd0"], P, n)
    gT = _loss_grad(S, states[-1][0])
    rq, rqd, _, _ = oracle.rollout_grad(S, B, S["q0"], S["qd0"], P, n, gT, np.zeros_like(gT))
    gq, gqd = ctx.rollout_backward(sc, P, _dev(S["q0"]), _dev(S["qd0"]), n, 4, _dev(gT), _dev(np.zeros_like(gT)),
                                   rtol=1e-13)
    np.testing.assert_allclose(gqd.cpu().numpy(), rqd, rtol=0, atol=1e-5 * np.abs(rqd).max())
    np.testing.assert_allclose(gq.cpu().numpy(), rq, rtol=0, atol=1e-5 * np.abs(rq).max())


def test_rollout_checkpoint_spacing_and_autograd(abd, ctx):
    S, P = sg.three_cubes()
    P = dict(P, pcg_rtol=1e-13, max_pcg=20000)
    S = dict(S)
    S["qd0"] = S["qd0"].copy()
    S["qd0"][1:, 1] = -0.5
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    n = 12
    q0, qd0 = _dev(S["q0"]), _dev(S["qd0"])
    gT = torch.zeros_like(q0)
    gT[1, :3] = 1.0
    z = torch.zeros_like(q0)
    ref = ctx.rollout_backward(sc, P, q0, qd0, n, 1, gT, z)
    for ck in (4, 5, 12, 20):
        got = ctx.rollout_backward(sc, P, q0, qd0, n, ck, gT, z)
        assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])
    # checkpoints kept by the forward rollout give the same gradient
    qf, qdf = q0.clone(), qd0.clone()
    ckp, nt = ctx.rollout_forward(sc, P, qf, qdf, n, 5)
    assert nt >= n
    got = ctx.rollout_backward(sc, P, q0, qd0, n, 5, gT, z, checkpoints=ckp)
    assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])
    assert torch.equal(ckp[-1, 0], qf) and torch.equal(ckp[-1, 1], qdf)
    # every state kept: no re-runs
    qf, qdf = q0.clone(), qd0.clone()
    ck1, _ = ctx.rollout_forward(sc, P, qf, qdf, n, 1)
    got = ctx.rollout_backward(sc, P, q0, qd0, n, 1, gT, z, checkpoints=ck1)
    assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])
    qa = q0.clone().requires_grad_(True)
    qda = qd0.clone().requires_grad_(True)
    qT, qdT = abd.rollout(ctx, sc, P, qa, qda, n, checkpoint_every=4)
    (qT[1, :3].sum()).backward()
    assert torch.equal(qa.grad, ref[0]) and torch.equal(qda.grad, ref[1])

"""The adjoint at the differentiable-rollout workload's size: 500
icospheres over the fixed box with lagged friction 0.5, taken at the
landing of the bottom layer (100 spheres within dhat of the floor, moving
down at 1 m/s), differentiated over a short horizon (5 steps, before the
pile's contacts make the trajectory chaotic).  Loss |p_1(T) - target|^2;
gradient with respect to all 500 x 12 initial velocities.

Checks: against central differences of the GPU rollout (h = 1e-6) along
20 seeded unit directions, 1e-5 of the gradient's norm; against the
oracle's adjoint on the same horizon, 1e-5 relative.  The rollouts stop
Newton where the last direction moves no vertex by more than 1e-8 m (well
above the floor of about 2e-10 m where FP64 energies stop decreasing), so
every perturbed rollout takes the same iterations and line-search steps
and the differences see a smooth map."""
import numpy as np
import pytest

import oracle
import scenegen as sg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N_STEPS = 5


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


def _setup():
    S, P, target = sg.adjoint_drop()
    S = sg.landed(S, seed=55, dhat=P["dhat"])
    P = dict(P, newton_tol=1e-6, pcg_rtol=1e-13, max_pcg=20000, max_newton=500)
    return S, P, target


def _loss(ctx, sc, P, q0, qd0, b1, target):
    q, qd = q0.clone(), qd0.clone()
    for _ in range(N_STEPS):
        st = ctx.time_step(sc, P, q, qd)
        assert st["converged"] == 1
    d = q[b1, :3] - target
    return float((d * d).sum()), q


def test_adjoint_drop_gradient(abd, ctx):
    S, P, target = _setup()
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    assert len(S["q0"]) == 501
    free = S["body_fixed"] == 0
    b1 = int(np.flatnonzero(free)[0])
    tq = _dev(target)
    q0, qd0 = _dev(S["q0"]), _dev(S["qd0"])
    L0, qT = _loss(ctx, sc, P, q0, qd0, b1, tq)
    gT = torch.zeros_like(q0)
    gT[b1, :3] = 2.0 * (qT[b1, :3] - tq)
    gq, gqd = ctx.rollout_backward(sc, P, q0, qd0, N_STEPS, N_STEPS, gT, torch.zeros_like(q0), rtol=1e-13)
    g = gqd.cpu().numpy()
    gn = np.linalg.norm(g)
    assert gn > 1e-3
    # central differences along 20 seeded unit directions over the free
    # bodies' velocities
    rng = np.random.default_rng(2024)
    h = 1e-6
    errs = []
    for k in range(20):
        d = rng.normal(size=g.shape) * free[:, None]
        d /= np.linalg.norm(d)
        dd = _dev(d)
        Lp, _ = _loss(ctx, sc, P, q0, qd0 + h * dd, b1, tq)
        Lm, _ = _loss(ctx, sc, P, q0, qd0 - h * dd, b1, tq)
        fd = (Lp - Lm) / (2.0 * h)
        errs.append(abs(fd - float((g * d).sum())) / gn)
    assert max(errs) <= 1e-5, errs
    # the oracle's adjoint of the same rollout
    B = oracle.Body(S)
    states, _ = oracle.rollout(S, B, S["q0"], S["qd0"], P, N_STEPS)
    qTo = states[-1][0]
    np.testing.assert_allclose(qT.cpu().numpy(), qTo, rtol=0, atol=1e-6)
    gTo = np.zeros_like(qTo)
    gTo[b1, :3] = 2.0 * (qTo[b1, :3] - target)
    rq, rqd, _, _ = oracle.rollout_grad(S, B, S["q0"], S["qd0"], P, N_STEPS, gTo, np.zeros_like(gTo))
    np.testing.assert_allclose(g, rqd, rtol=0, atol=1e-5 * np.abs(rqd).max())
    np.testing.assert_allclose(gq.cpu().numpy(), rq, rtol=0, atol=1e-5 * np.abs(rq).max())

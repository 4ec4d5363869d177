"""GPU parity on the wrecking-ball-shaped workload (570 bodies: a wall of
560 cubes resting within dhat of their supports, a chain of stadium links
from a fixed pivot, and a ball with an eyelet ring on the last link; the
shape of the paper's wrecking-ball scene, sec. 5, Tab. tab:time).

At full size from the generator's state: static candidates bit-exact, the
barrier gradient and projected Hessian blocks within 1e-10 (tens of
thousands of resting pairs, many nearly parallel edges under the
mollifier); the swept candidates and CCD bound of one step of a ball moving
at 3 m/s into the wall; one Newton step within 1e-8 of the oracle's; three
time steps of the swinging chain and settling wall within 1e-6."""
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


def test_wrecking_ball_barrier_and_ccd(abd, ctx):
    S, P = sg.wrecking_ball()
    assert len(S["q0"]) == 570
    sc = abd.Scene(S)
    x = oracle.vertex_map(S, S["q0"])
    pt, ee = oracle.candidates(S, x, None, P["dhat"])
    gpt, gee = ctx.candidates(sc, _dev(x), None, P["dhat"])
    np.testing.assert_array_equal(_sorted(gpt.cpu().numpy()), pt)
    np.testing.assert_array_equal(_sorted(gee.cpu().numpy()), ee)
    keys = oracle.off_keys(S, pt, ee)
    np.testing.assert_array_equal(ctx.offdiag_pattern(sc, gpt, gee).cpu().numpy(), keys)
    r, gs, Ds, Os = abs_scale(S, x, pt, ee, P, keys)
    assert r["n_active"] > 10000 and len(keys) > 500
    e, g, D, O = ctx.barrier_grad_hess(sc, P, _dev(x), _dev(pt, torch.int32), _dev(ee, torch.int32),
                                       _dev(keys, torch.int32))
    assert abs(e.item() - r["energy"]) <= 1e-10 * abs(r["energy"])
    worst = lambda a, b, s: float(np.max(np.abs(a - b) / np.maximum(s, 1e-300)))
    errs = dict(g=worst(g.cpu().numpy(), r["grad"], gs), D=worst(D.cpu().numpy(), r["diag"], Ds),
                O=worst(O.cpu().numpy(), r["off"], Os))
    assert max(errs.values()) <= 1e-10, errs
    # the ball 1 cm from the wall moving into it at 3 m/s for one step
    q1 = S["q0"].copy()
    ball = len(q1) - 1
    q0 = S["q0"].copy()
    sl = slice(S["body_vert_off"][ball], S["body_vert_off"][ball + 1])
    front = (S["xbar"][sl] @ q0[ball, 3:].reshape(3, 3).T)[:, 0].max()
    q0[ball, 0] += 0.27 - 0.01 - (q0[ball, 0] + front)
    q0[ball, 1] = 1.0
    q1 = q0.copy()
    q1[ball, 0] += 3.0 * P["dt"]
    x0, x1 = oracle.vertex_map(S, q0), oracle.vertex_map(S, q1)
    spt, see = oracle.candidates(S, x0, x1, P["dhat"])
    gspt, gsee = ctx.candidates(sc, _dev(x0), _dev(x1), P["dhat"])
    np.testing.assert_array_equal(_sorted(gspt.cpu().numpy()), spt)
    np.testing.assert_array_equal(_sorted(gsee.cpu().numpy()), see)
    tp, te, alpha = ctx.ccd_max_step(sc, P, _dev(x0), _dev(x1 - x0), _dev(spt, torch.int32), _dev(see, torch.int32))
    otp, ote, oalpha = oracle.ccd(S, x0, x1 - x0, spt, see, P)
    for t, ot in ((tp.cpu().numpy(), otp), (te.cpu().numpy(), ote)):
        assert np.all(t <= ot * (1 + 1e-9)) and np.all(t >= 0.99 * ot)
    assert oalpha < 0.5
    assert oalpha * 0.99 <= alpha.item() <= oalpha * (1 + 1e-9)


def test_wrecking_ball_newton_and_steps(abd, ctx):
    S, P = sg.wrecking_ball()
    P = dict(P, newton_tol=1e-5, pcg_rtol=1e-14, max_pcg=50000)
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    B = oracle.Body(S)
    q, qd = S["q0"].copy(), S["qd0"].copy()
    qt = oracle.q_tilde(S, q, qd, P)
    qn_ref, conv, info = oracle.newton_iteration(S, B, q, qt, P)
    assert not conv and info["n_active"] > 10000
    qg = _dev(q)
    st = ctx.newton_step(sc, P, qg, _dev(qt))
    assert st["n_active_pt"] + st["n_active_ee"] == info["n_active"]
    assert st["alpha"] == pytest.approx(info["alpha"], rel=1e-9)
    ref = qn_ref - q
    err = np.abs(qg.cpu().numpy() - q - ref).max() / np.abs(ref).max()
    assert err <= 1e-8, err
    P = dict(P, pcg_rtol=1e-13)
    qg, qdg = _dev(q), _dev(qd)
    for step in range(3):
        q, qd, its = oracle.time_step(S, B, q, qd, P)
        st = ctx.time_step(sc, P, qg, qdg)
        assert st["converged"] == 1
        np.testing.assert_allclose(qg.cpu().numpy(), q, rtol=0, atol=1e-6)

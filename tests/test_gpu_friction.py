"""GPU parity of the lagged friction path (friction potential of the
incremental potential, sec. 4) against the CPU oracle on identical seeded
inputs.  Bars: the lagged set (lambda > 0) bit-exact; lambda 1e-10 relative;
closest-point weights 1e-8 absolute (they lie in [-1, 1]); the tangent plane
compared through its projector T T^T (the basis inside the plane is a
convention: the friction energy depends only on the projector) to 1e-9;
energies 1e-10 relative; gradients and Hessian blocks 1e-10 of the largest
entry; Newton steps 1e-8."""
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


def _scenes():
    out = []
    for seed in range(3):
        S = sg.near_contact_cubes(seed, n=4)
        out.append((f"cubes{seed}", S, sg.default_params(dhat=1e-3, kappa_b=80.0, mu=0.4)))
    S = sg.triangle_soup(7, n_bodies=16, extent=4e-3, tri_size=5e-3)
    out.append(("soup", S, sg.default_params(dhat=1e-3, kappa_b=1.0, mu=0.3)))
    return out


SCENES = _scenes()


def _state(S, seed):
    return sg.random_state(S, seed, rot_angle=2e-4, stretch=1e-5, shift=1e-4)


def _slide(S, q, seed, scale, eps):
    """q with every free body translated tangentially by scale * eps and a
    tiny random affine change."""
    rng = np.random.default_rng(seed)
    q = q.copy()
    for b in np.flatnonzero(S["body_fixed"] == 0):
        d = rng.normal(size=3)
        d[1] = 0.0
        q[b, :3] += scale * eps * d / np.linalg.norm(d)
        q[b, 3:] += rng.normal(size=9) * 1e-8
    return q


def _lag_both(ctx, sc, S, P, xt):
    pt, ee = oracle.candidates(S, xt, None, P["dhat"])
    F = oracle.friction_lag(S, xt, pt, ee, P, keep_inactive=True)
    lam, T, w = ctx.friction_lag(sc, P, _dev(xt), _dev(pt, torch.int32), _dev(ee, torch.int32))
    return pt, ee, F, lam.cpu().numpy(), T.cpu().numpy(), w.cpu().numpy()


@pytest.mark.parametrize("name,S,P", SCENES, ids=[s[0] for s in SCENES])
def test_friction_lag_parity(abd, ctx, name, S, P):
    sc = abd.Scene(S)
    n_act = 0
    for seed in (1, 2):
        xt = oracle.vertex_map(S, _state(S, seed))
        pt, ee, F, lam, T, w = _lag_both(ctx, sc, S, P, xt)
        rl = np.concatenate([F["pt"]["lam"], F["ee"]["lam"]])
        rT = np.concatenate([F["pt"]["T"], F["ee"]["T"]])
        rw = np.concatenate([F["pt"]["w"], F["ee"]["w"]])
        np.testing.assert_array_equal(lam > 0, rl > 0)
        act = rl > 0
        n_act += int(act.sum())
        np.testing.assert_allclose(lam, rl, rtol=1e-10, atol=0)
        np.testing.assert_allclose(w[act], rw[act], rtol=0, atol=1e-8)
        np.testing.assert_array_equal(w[~act], 0.0)
        Pg = np.einsum("nai,naj->nij", T.reshape(-1, 2, 3), T.reshape(-1, 2, 3))
        Pr = np.einsum("nai,naj->nij", rT.reshape(-1, 2, 3), rT.reshape(-1, 2, 3))
        np.testing.assert_allclose(Pg[act], Pr[act], rtol=0, atol=1e-9)
    assert n_act > 0


@pytest.mark.parametrize("scale", [0.3, 3.0])
@pytest.mark.parametrize("name,S,P", SCENES, ids=[s[0] for s in SCENES])
def test_friction_grad_hess_parity(abd, ctx, name, S, P, scale):
    sc = abd.Scene(S)
    q0 = _state(S, 5)
    xt = oracle.vertex_map(S, q0)
    pt, ee = oracle.candidates(S, xt, None, P["dhat"])
    F = oracle.friction_lag(S, xt, pt, ee, P)
    fpt, fee = F["pt"]["pairs"], F["ee"]["pairs"]
    assert len(fpt) + len(fee) > 0
    keys = oracle.off_keys(S, fpt, fee)
    eps = P["eps_v"] * P["dt"]
    x = oracle.vertex_map(S, _slide(S, q0, 9, scale, eps))
    r = oracle.friction(S, x, F, P, keys)
    lam = np.concatenate([F["pt"]["lam"], F["ee"]["lam"]])
    T = np.concatenate([F["pt"]["T"], F["ee"]["T"]])
    w = np.concatenate([F["pt"]["w"], F["ee"]["w"]])
    args = (_dev(x), _dev(xt), _dev(fpt, torch.int32), _dev(fee, torch.int32), _dev(lam), _dev(T), _dev(w))
    e, g, D, O = ctx.friction_grad_hess(sc, P, *args, _dev(keys, torch.int32))
    assert e.item() == pytest.approx(r["energy"], rel=1e-10)
    gs = np.abs(r["grad"]).max()
    hs = max(np.abs(r["diag"]).max(), np.abs(r["off"]).max() if len(keys) else 0.0)
    np.testing.assert_allclose(g.cpu().numpy(), r["grad"], rtol=0, atol=1e-10 * gs)
    np.testing.assert_allclose(D.cpu().numpy(), r["diag"], rtol=0, atol=1e-10 * hs)
    if len(keys):
        np.testing.assert_allclose(O.cpu().numpy(), r["off"], rtol=0, atol=1e-10 * hs)
    eo = ctx.friction_energy(sc, P, *args).item()
    assert eo == pytest.approx(r["energy"], rel=1e-10)


def test_friction_inactive_and_empty_inputs(abd, ctx):
    # pairs with lambda = 0 contribute nothing; empty pair lists are valid
    S, P = SCENES[0][1], SCENES[0][2]
    sc = abd.Scene(S)
    xt = oracle.vertex_map(S, _state(S, 3))
    pt, ee, F, lam, T, w = _lag_both(ctx, sc, S, P, xt)
    keys = oracle.off_keys(S, pt, ee)
    x = oracle.vertex_map(S, _slide(S, _state(S, 3), 4, 2.0, 1e-5))
    args = (_dev(x), _dev(xt), _dev(pt, torch.int32), _dev(ee, torch.int32))
    e_all, g_all, D_all, O_all = ctx.friction_grad_hess(sc, P, *args, _dev(lam), _dev(T), _dev(w),
                                                        _dev(keys, torch.int32))
    act = lam > 0
    npt = len(pt)
    Fk = dict(pt=dict(pairs=pt[act[:npt]], lam=lam[:npt][act[:npt]], T=T[:npt][act[:npt]], w=w[:npt][act[:npt]]),
              ee=dict(pairs=ee[act[npt:]], lam=lam[npt:][act[npt:]], T=T[npt:][act[npt:]], w=w[npt:][act[npt:]]),
              xt=xt)
    r = oracle.friction(S, x, Fk, P, keys)
    assert e_all.item() == pytest.approx(r["energy"], rel=1e-10)
    np.testing.assert_allclose(g_all.cpu().numpy(), r["grad"], rtol=0, atol=1e-10 * np.abs(r["grad"]).max())
    z = np.zeros((0, 2), np.int32)
    e0, g0, _, _ = ctx.friction_grad_hess(sc, P, _dev(x), _dev(xt), _dev(z, torch.int32), _dev(z, torch.int32),
                                          _dev(np.zeros(0)), _dev(np.zeros((0, 6))), _dev(np.zeros((0, 4))),
                                          _dev(keys, torch.int32))
    assert e0.item() == 0.0 and float(g0.abs().max()) == 0.0


@pytest.mark.parametrize("name,S,P", SCENES[:3], ids=[s[0] for s in SCENES[:3]])
def test_newton_step_with_friction_parity(abd, ctx, name, S, P):
    P = dict(P, pcg_rtol=1e-14, max_pcg=20000)
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    B = oracle.Body(S)
    q = _state(S, 61)
    qd = np.zeros_like(q)
    free = S["body_fixed"] == 0
    qd[free, 1] = -0.05
    qd[free, 0] = 0.02
    qd[free, 2] = -0.03
    qt = oracle.q_tilde(S, q, qd, P)
    F = oracle.step_friction(S, q, P)
    n_ref = len(F["pt"]["pairs"]) + len(F["ee"]["pairs"])
    assert n_ref > 0
    qn_ref, conv_ref, info = oracle.newton_iteration(S, B, q, qt, P, F)
    qg = _dev(q)
    n_fr = ctx.friction_begin_step(sc, P, qg)
    try:
        st = ctx.newton_step(sc, P, qg, _dev(qt))
    finally:
        ctx.friction_end_step()
    assert n_fr == n_ref and st["n_friction"] == n_ref
    assert bool(st["converged"]) == conv_ref
    if not conv_ref:
        assert st["alpha"] == pytest.approx(info["alpha"], rel=1e-2)
        ref = qn_ref - q
        dq = qg.cpu().numpy() - q
        assert np.abs(dq - ref).max() <= 1e-8 * np.abs(ref).max()
    assert st["disp"] == pytest.approx(info["disp"], rel=1e-6)


def test_time_steps_slope_trajectory_and_closed_form(abd, ctx):
    # the GPU time step on the inclined plane follows the oracle and the
    # Coulomb closed form a = g (sin t - mu cos t)
    theta, mu = math.atan(0.75), 0.5
    S, P = sg.cube_on_slope(theta, mu, v0=1.0)
    P = dict(P, pcg_rtol=1e-13, max_pcg=20000)
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    B = oracle.Body(S)
    q, qd = S["q0"].copy(), S["qd0"].copy()
    qg, qdg = _dev(q), _dev(qd)
    vs = []
    for step in range(30):
        q, qd, its = oracle.time_step(S, B, q, qd, P)
        st = ctx.time_step(sc, P, qg, qdg)
        assert st["converged"] == 1 and st["n_friction"] > 0
        np.testing.assert_allclose(qg.cpu().numpy(), q, rtol=0, atol=1e-6)
        vs.append(qdg[1, 0].item())
    a = (vs[-1] - vs[10]) / ((len(vs) - 1 - 10) * P["dt"])
    assert a == pytest.approx(9.8 * (math.sin(theta) - mu * math.cos(theta)), rel=1e-3)

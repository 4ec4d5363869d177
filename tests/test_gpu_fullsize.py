"""GPU parity at the sizes the solver and the Newton driver are timed at:
states with hundreds of solver blocks and rows of up to 26 off-diagonal
body blocks, so that the PCG's cross-block fold, its multi-pass entry loop
and the multi-block line-search reductions are compared with the oracle.

Scenes (positions only, from the seeded generators): a 10x10x10 lattice of
cubes with every interior cube within dhat of its 26 neighbours (900 free
bodies, 225 solver blocks of 4 bodies), and 1000 icospheres packed face-
centred cubic (950 free bodies, 12 neighbours each).

Bars as for the small scenes: barrier gradient and projected Hessian blocks
(diagonal and off-diagonal) 1e-10 against the summation-order-invariant
scale; PCG at rtol 1e-14 within 1e-8 of the oracle's direct solve; the
Newton step within 1e-8 of the oracle's; a time step at the benchmark's own
inexact settings (PCG rtol 1e-2, Newton tolerance 1e-2 of the box diagonal
per second) within the bound those settings give (below)."""
import numpy as np
import pytest

import oracle
import scenegen as sg
from parity_scales import abs_scale as _abs_scale

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SWBB = 4  # bodies per solver block


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


_CACHE = {}


def _scene(name):
    """Scene, params, state, q~ and the oracle's gradient/Hessian there
    (computed once per module run)."""
    if name in _CACHE:
        return _CACHE[name]
    S, P = sg.cube_lattice() if name == "lattice" else sg.icosphere_fcc()
    B = oracle.Body(S)
    q = S["q0"].copy()
    qd = np.zeros_like(q)
    qd[S["body_fixed"] == 0, 1] = -0.05
    qt = oracle.q_tilde(S, q, qd, P)
    x = oracle.vertex_map(S, q)
    pt, ee = oracle.candidates(S, x, None, P["dhat"])
    gh = oracle.grad_hess(S, B, q, qt, P, x=x, pt=pt, ee=ee)
    _CACHE[name] = (S, P, B, q, qt, x, gh)
    return _CACHE[name]


def _structure(S, keys):
    """Solver blocks and the largest number of off-diagonal blocks in one
    body's row (free bodies only)."""
    free = S["body_fixed"] == 0
    cnt = np.zeros(len(free), np.int64)
    for a, b in keys:
        if free[a] and free[b]:
            cnt[a] += 1
            cnt[b] += 1
    return (int(free.sum()) + SWBB - 1) // SWBB, int(cnt.max())


@pytest.mark.parametrize("name", ["lattice", "fcc"])
def test_barrier_offdiag_blocks_full_size(abd, ctx, name):
    S, P, B, q, qt, x, gh = _scene(name)
    pt, ee, keys = gh["pt"], gh["ee"], gh["keys"]
    nblocks, max_row = _structure(S, keys)
    assert nblocks >= 200 and max_row > 10 and len(keys) > 4000
    sc = abd.Scene(S)
    # candidates bit-exact at full size
    gpt, gee = ctx.candidates(sc, _dev(x), None, P["dhat"])
    srt = lambda a: a[np.lexsort((a[:, 1], a[:, 0]))] if len(a) else a
    np.testing.assert_array_equal(srt(gpt.cpu().numpy().astype(np.int64)), pt)
    np.testing.assert_array_equal(srt(gee.cpu().numpy().astype(np.int64)), ee)
    np.testing.assert_array_equal(ctx.offdiag_pattern(sc, gpt, gee).cpu().numpy(), keys)
    r, gs, Ds, Os = _abs_scale(S, x, pt, ee, P, keys)
    assert r["n_active"] > 5000
    e, g, D, O = ctx.barrier_grad_hess(sc, P, _dev(x), _dev(pt, torch.int32), _dev(ee, torch.int32),
                                       _dev(keys, torch.int32))
    tol = 1e-10
    assert abs(e.item() - r["energy"]) <= tol * abs(r["energy"])

    def worst(a, b, s):
        return float(np.max(np.abs(a - b) / np.maximum(s, 1e-300)))

    errs = dict(g=worst(g.cpu().numpy(), r["grad"], gs), D=worst(D.cpu().numpy(), r["diag"], Ds),
                O=worst(O.cpu().numpy(), r["off"], Os))
    assert max(errs.values()) <= tol, errs
    # the off-diagonal blocks carry real coupling
    assert np.abs(r["off"]).max() > 1e-3 * np.abs(r["diag"]).max()


@pytest.mark.parametrize("name", ["lattice", "fcc"])
def test_pcg_full_size_matches_direct_solve(abd, ctx, name):
    S, P, B, q, qt, x, gh = _scene(name)
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    p_ref = oracle.solve(S, gh["diag"], gh["off"], gh["keys"], -gh["grad"])
    p, its = ctx.pcg_solve(sc, _dev(gh["diag"]), _dev(gh["off"]), _dev(gh["keys"], torch.int32),
                           _dev(-gh["grad"]), rtol=1e-14, max_iter=50000)
    assert its > 20
    err = np.abs(p.cpu().numpy() - p_ref).max() / np.abs(p_ref).max()
    assert err <= 1e-8, err


@pytest.mark.parametrize("name", ["lattice", "fcc"])
def test_newton_step_full_size(abd, ctx, name):
    S, P, B, q, qt, x, gh = _scene(name)
    P = dict(P, pcg_rtol=1e-14, max_pcg=50000)
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    qn_ref, conv_ref, info = oracle.newton_iteration(S, B, q, qt, P)
    assert not conv_ref
    qg = _dev(q)
    st = ctx.newton_step(sc, P, qg, _dev(qt))
    assert not st["converged"]
    assert st["n_active_pt"] + st["n_active_ee"] == info["n_active"]
    assert st["n_pt_swept"] == info["n_pt_swept"] and st["n_ee_swept"] == info["n_ee_swept"]
    assert st["alpha"] == pytest.approx(info["alpha"], rel=1e-9)
    ref = qn_ref - q
    dq = qg.cpu().numpy() - q
    err = np.abs(dq - ref).max() / np.abs(ref).max()
    assert err <= 1e-8, err


def test_time_step_benchmark_settings_landing(abd, ctx):
    """One time step at the benchmark's inexact settings: the bottom layer
    of the icosphere box (100 spheres resting within dhat of the floor)
    hit at 1 m/s, lagged friction mu 0.5.  Each side stops when its last
    Newton direction moves no vertex by more than tol_v dt; to first order
    that direction is the distance to the step's minimiser, so the two
    results differ by at most about 2 tol_v dt per vertex (the GPU's
    direction is inexact by the PCG tolerance, a relative 1e-2)."""
    S, P = sg.icosphere_resting_layer()
    assert P["pcg_rtol"] == 1e-2 and P["mu"] == 0.5
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    B = oracle.Body(S)
    q, qd = S["q0"].copy(), S["qd0"].copy()
    qd[S["body_fixed"] == 0, 1] = -1.0
    qg, qdg = _dev(q), _dev(qd)
    for step in range(2):
        q, qd, its = oracle.time_step(S, B, q, qd, P)
        st = ctx.time_step(sc, P, qg, qdg)
        assert st["converged"] == 1
        bound = 2.0 * (1.0 + P["pcg_rtol"]) * P["newton_tol"] * P["dt"]
        xg = oracle.vertex_map(S, qg.cpu().numpy())
        xo = oracle.vertex_map(S, q)
        dx = np.abs(xg - xo).max()
        assert dx <= bound, (step, dx, bound)
        q, qd = qg.cpu().numpy(), qdg.cpu().numpy()  # continue both from the GPU's state
    # the spheres were stopped by the floor (y = 0), not passed through it
    free = S["body_fixed"][S["vert_body"]] == 0
    assert oracle.vertex_map(S, qg.cpu().numpy())[free, 1].min() > 0.0

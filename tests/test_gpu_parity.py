"""GPU parity: every ABI call of the HIP library against the CPU oracle on
identical seeded inputs.  Bars: bit-exact for sets, codes and the vertex
map; 1e-10 relative (per entry, against the sum of absolute pair
contributions) for barrier gradients and Hessians; Newton steps 1e-8;
CCD bounds conservative and within 1% of the oracle's."""
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


def _sorted_pairs(a):
    a = np.asarray(a, dtype=np.int64).reshape(-1, 2)
    if len(a) == 0:
        return a
    return a[np.lexsort((a[:, 1], a[:, 0]))]


def _scenes():
    out = []
    for seed in range(3):
        S = sg.near_contact_cubes(seed, n=4)
        out.append((f"cubes{seed}", S, sg.default_params(dhat=1e-3, kappa_b=80.0)))
    S = sg.triangle_soup(7, n_bodies=16, extent=4e-3, tri_size=5e-3)
    out.append(("soup", S, sg.default_params(dhat=1e-3, kappa_b=1.0)))
    S, P = sg.three_cubes()
    out.append(("three_cubes", S, P))
    return out


SCENES = _scenes()


def _state(S, seed):
    return sg.random_state(S, seed, rot_angle=2e-4, stretch=1e-5, shift=1e-4)


# ------------------------------------------------------------- a1, mass ----

@pytest.mark.parametrize("name,S,P", SCENES, ids=[s[0] for s in SCENES])
def test_vertex_map_bit_exact(abd, ctx, name, S, P):
    sc = abd.Scene(S)
    for seed in range(3):
        q = sg.random_state(S, seed, rot_angle=1.0, stretch=0.1, shift=0.3)
        x = ctx.vertex_map(sc, _dev(q)).cpu().numpy()
        np.testing.assert_array_equal(x, oracle.vertex_map(S, q))


def test_vertex_map_full_size_icosphere_box(abd, ctx):
    S, P = sg.icosphere_box()
    sc = abd.Scene(S)
    q = sg.random_state(S, 3, rot_angle=0.5, stretch=1e-3, shift=0.01)
    x = ctx.vertex_map(sc, _dev(q)).cpu().numpy()
    np.testing.assert_array_equal(x, oracle.vertex_map(S, q))


@pytest.mark.parametrize("name,S,P", SCENES, ids=[s[0] for s in SCENES])
def test_body_mass(abd, ctx, name, S, P):
    sc = abd.Scene(S)
    m, v = ctx.body_mass(sc)
    om, ov = oracle.mass_properties(S)
    np.testing.assert_allclose(m.cpu().numpy(), om, rtol=1e-13, atol=1e-13 * np.abs(om).max())
    np.testing.assert_allclose(v.cpu().numpy(), ov, rtol=1e-13, atol=1e-16)


# ------------------------------------------------------ a2 candidates ----

@pytest.mark.parametrize("name,S,P", SCENES, ids=[s[0] for s in SCENES])
def test_candidates_bit_exact(abd, ctx, name, S, P):
    sc = abd.Scene(S)
    q0 = _state(S, 1)
    q1 = sg.random_state(S, 2, rot_angle=1e-3, shift=2e-3)
    x0 = oracle.vertex_map(S, q0)
    x1 = oracle.vertex_map(S, q1)
    for a, b in ((x0, None), (x0, x1)):
        pt, ee = ctx.candidates(sc, _dev(a), None if b is None else _dev(b), P["dhat"])
        opt, oee = oracle.candidates(S, a, b, P["dhat"])
        np.testing.assert_array_equal(_sorted_pairs(pt.cpu().numpy()), opt)
        np.testing.assert_array_equal(_sorted_pairs(ee.cpu().numpy()), oee)
        # keys
        keys = ctx.offdiag_pattern(sc, pt, ee).cpu().numpy()
        np.testing.assert_array_equal(keys, oracle.off_keys(S, opt, oee))


def test_candidates_grouped_order(abd, ctx):
    S = sg.near_contact_cubes(4, n=5)
    sc = abd.Scene(S)
    x = oracle.vertex_map(S, S["q0"])
    pt, ee = ctx.candidates(sc, _dev(x), None, 1e-3)
    pt = pt.cpu().numpy()
    b = np.stack([S["vert_body"][pt[:, 0]], S["tri_body"][pt[:, 1]]], 1)
    key = np.minimum(b[:, 0], b[:, 1]) * 10000 + np.maximum(b[:, 0], b[:, 1])
    assert np.all(np.diff(key) >= 0)


def test_candidates_capacity_error(abd, ctx):
    S = sg.near_contact_cubes(0, n=3)
    sc = abd.Scene(S)
    x = _dev(oracle.vertex_map(S, S["q0"]))
    with pytest.raises(abd.AbdError) as ei:
        _cap_call(abd, ctx, sc, x)
    assert "CAPACITY" in str(ei.value)


def _cap_call(abd, ctx, sc, x):
    import ctypes
    pt = torch.empty((1, 2), dtype=torch.int32, device="cuda:0")
    ee = torch.empty((1, 2), dtype=torch.int32, device="cuda:0")
    npt, nee = ctypes.c_int64(0), ctypes.c_int64(0)
    rc = ctx.L.abd_candidates(ctx.h, ctypes.byref(sc.c), abd._ptr(x), None, 1e-3, abd._ptr(pt), 1,
                              ctypes.byref(npt), abd._ptr(ee), 1, ctypes.byref(nee), abd._stream())
    assert npt.value > 1 and nee.value > 1
    ctx._check(rc)


def test_candidates_full_size_swept_icosphere_box(abd, ctx):
    S, P = sg.icosphere_box()
    sc = abd.Scene(S)
    q0 = S["q0"].copy()
    q1 = q0.copy()
    q1[1:101, 1] -= 0.25  # the lowest layer sweeps through the floor
    q1[101:, 1] -= 0.02
    x0, x1 = oracle.vertex_map(S, q0), oracle.vertex_map(S, q1)
    pt, ee = ctx.candidates(sc, _dev(x0), _dev(x1), P["dhat"])
    opt, oee = oracle.candidates(S, x0, x1, P["dhat"])
    assert len(opt) > 1000
    np.testing.assert_array_equal(_sorted_pairs(pt.cpu().numpy()), opt)
    np.testing.assert_array_equal(_sorted_pairs(ee.cpu().numpy()), oee)


# ---------------------------------------------------- a3 narrow phase ----

@pytest.mark.parametrize("name,S,P", SCENES, ids=[s[0] for s in SCENES])
def test_classify_bit_exact(abd, ctx, name, S, P):
    sc = abd.Scene(S)
    x = oracle.vertex_map(S, _state(S, 5))
    pt, ee = oracle.candidates(S, x, None, 10 * P["dhat"])
    for is_ee, pairs in ((0, pt), (1, ee)):
        if len(pairs) == 0:
            continue
        ty, d2, act = ctx.classify(sc, _dev(x), _dev(pairs, torch.int32), is_ee, P["dhat"])
        oty, od2, oact = oracle.classify(S, x, pairs, is_ee, P["dhat"])
        np.testing.assert_array_equal(ty.cpu().numpy(), oty)
        np.testing.assert_array_equal(d2.cpu().numpy(), od2)
        np.testing.assert_array_equal(act.cpu().numpy(), oact)


def test_classify_random_primitives_all_cases(abd, ctx):
    # random vertex soups exercise every case code on both sides
    rng = np.random.default_rng(77)
    n = 20000
    X = rng.normal(size=(4 * n, 3))
    b = sg.SceneBuilder()
    b.add(np.zeros((3, 3)), np.array([[0, 1, 2]], np.int32))
    S = b.build()
    S = dict(S, tris=np.arange(4 * n, dtype=np.int32).reshape(n, 4)[:, 1:].copy(),
             edges=np.arange(4 * n, dtype=np.int32).reshape(2 * n, 2).copy())
    sc = abd.Scene(S)
    pt = np.stack([np.arange(n) * 4, np.arange(n)], 1).astype(np.int32)
    ee = np.stack([np.arange(n) * 2, np.arange(n) * 2 + 1], 1).astype(np.int32)
    for is_ee, pairs in ((0, pt), (1, ee)):
        ty, d2, act = ctx.classify(sc, _dev(X), _dev(pairs, torch.int32), is_ee, 1.0)
        oty, od2, oact = oracle.classify(S, X, pairs, is_ee, 1.0)
        np.testing.assert_array_equal(ty.cpu().numpy(), oty)
        np.testing.assert_array_equal(d2.cpu().numpy(), od2)
        np.testing.assert_array_equal(act.cpu().numpy(), oact)
        assert len(np.unique(oty)) >= (9 if is_ee else 7)


# ------------------------------------------- a4-a6 barrier assembly ----

def _abs_scale(S, x, pt, ee, P, keys):
    """Summation-order-invariant tolerance scales: gradients per entry
    sum_pairs |J|^T |g_loc|; Hessians per entry sum_pairs |H_pair|_max
    (|J|^T 1 |J|), the normwise error bound of a backward-stable symmetric
    eigensolver (error ~ eps |H| for every entry of the projected matrix)
    carried through the fixed J^T H J maps."""
    r = oracle.barrier(S, x, pt, ee, P, keys, project=True, local=True)
    ru = oracle.barrier(S, x, pt, ee, P, keys, project=False, local=True)
    nb = len(S["body_fixed"])
    gs = np.zeros((nb, 12))
    Ds = np.zeros((nb, 144))
    Os = np.zeros((len(keys), 144))
    kmap = {(int(a), int(b)): i for i, (a, b) in enumerate(keys)}

    def Jv(v):
        J = np.zeros((3, 12))
        J[:, :3] = np.eye(3)
        for i in range(3):
            J[i, 3 + 3 * i:6 + 3 * i] = S["xbar"][v]
        return J

    for name, pairs in (("pt", pt), ("ee", ee)):
        lg, lH = r["local"][name]
        _, lHu = ru["local"][name]
        for i, pr in enumerate(pairs):
            if not np.any(lHu[i]):
                continue
            vid = [pr[0], *S["tris"][pr[1]]] if name == "pt" else [*S["edges"][pr[0]], *S["edges"][pr[1]]]
            bod = [S["vert_body"][v] for v in vid]
            H = np.full((12, 12), max(np.abs(lHu[i]).max(), np.abs(lH[i]).max()))
            for k in range(4):
                bk = bod[k]
                if S["body_fixed"][bk]:
                    continue
                gs[bk] += np.abs(Jv(vid[k])).T @ np.abs(lg[i][3 * k:3 * k + 3])
                for l in range(4):
                    bl = bod[l]
                    if S["body_fixed"][bl]:
                        continue
                    blk = np.abs(Jv(vid[k])).T @ H[3 * k:3 * k + 3, 3 * l:3 * l + 3] @ np.abs(Jv(vid[l]))
                    if bk == bl:
                        Ds[bk] += blk.reshape(144)
                    elif bk < bl:
                        Os[kmap[(bk, bl)]] += blk.reshape(144)
    return r, gs, Ds, Os


@pytest.mark.parametrize("name,S,P", SCENES, ids=[s[0] for s in SCENES])
def test_barrier_grad_hess_parity(abd, ctx, name, S, P):
    sc = abd.Scene(S)
    for seed in (11, 12):
        x = oracle.vertex_map(S, _state(S, seed))
        pt, ee = oracle.candidates(S, x, None, P["dhat"])
        keys = oracle.off_keys(S, pt, ee)
        r, gs, Ds, Os = _abs_scale(S, x, pt, ee, P, keys)
        if r["n_active"] == 0:
            continue
        e, g, D, O = ctx.barrier_grad_hess(sc, P, _dev(x), _dev(pt, torch.int32), _dev(ee, torch.int32),
                                           _dev(keys, torch.int32))
        tol = 1e-10
        assert abs(e.item() - r["energy"]) <= tol * abs(r["energy"]) + 1e-300

        def worst(a, b, scale):
            return float(np.max(np.abs(a - b) / np.maximum(scale, 1e-300)))

        errs = dict(g=worst(g.cpu().numpy(), r["grad"], gs), D=worst(D.cpu().numpy(), r["diag"], Ds))
        if len(keys):
            errs["O"] = worst(O.cpu().numpy(), r["off"], Os)
        assert max(errs.values()) <= tol, errs


def test_barrier_and_ccd_full_size_icosphere_box(abd, ctx):
    # the benchmark scene at full size (1000 icospheres, 162k vertices) with
    # its bottom layer lowered to rest U[0.2,0.8] dhat above the floor:
    # candidates (bit-exact), the assembled barrier gradient and projected
    # Hessian, and the CCD bound of a 4 mm downward sweep, against the oracle
    S, P = sg.icosphere_box()
    q = S["q0"].copy()
    rng = np.random.default_rng(123)
    for b in range(1, 101):
        sl = slice(S["body_vert_off"][b], S["body_vert_off"][b + 1])
        low = (S["xbar"][sl] @ q[b, 3:].reshape(3, 3).T)[:, 1].min()
        q[b, 1] = rng.uniform(0.2, 0.8) * P["dhat"] - low
    sc = abd.Scene(S)
    x = oracle.vertex_map(S, q)
    pt, ee = ctx.candidates(sc, _dev(x), _dev(x), P["dhat"])
    opt, oee = oracle.candidates(S, x, None, P["dhat"])
    np.testing.assert_array_equal(_sorted_pairs(pt.cpu().numpy()), opt)
    np.testing.assert_array_equal(_sorted_pairs(ee.cpu().numpy()), oee)
    keys = oracle.off_keys(S, opt, oee)
    r, gs, Ds, Os = _abs_scale(S, x, opt, oee, P, keys)
    assert r["n_active"] > 100  # (floor contacts only: no off-diagonal blocks at this state)
    e, g, D, O = ctx.barrier_grad_hess(sc, P, _dev(x), _dev(opt, torch.int32), _dev(oee, torch.int32),
                                       _dev(keys, torch.int32))
    tol = 1e-10
    assert abs(e.item() - r["energy"]) <= tol * abs(r["energy"])
    worst = lambda a, b, sc_: float(np.max(np.abs(a - b) / np.maximum(sc_, 1e-300)))
    errs = dict(g=worst(g.cpu().numpy(), r["grad"], gs), D=worst(D.cpu().numpy(), r["diag"], Ds))
    if len(keys):
        errs["O"] = worst(O.cpu().numpy(), r["off"], Os)
    assert max(errs.values()) <= tol, errs
    q1 = q.copy()
    q1[1:, 1] -= 4e-3
    x1 = oracle.vertex_map(S, q1)
    spt, see = oracle.candidates(S, x, x1, P["dhat"])
    tp, te, alpha = ctx.ccd_max_step(sc, P, _dev(x), _dev(x1 - x), _dev(spt, torch.int32), _dev(see, torch.int32))
    otp, ote, oalpha = oracle.ccd(S, x, x1 - x, spt, see, P)
    assert len(spt) + len(see) > 1000
    for t, ot in ((tp.cpu().numpy(), otp), (te.cpu().numpy(), ote)):
        assert np.all(t <= ot * (1 + 1e-9))
        assert np.all(t >= 0.99 * ot)
    assert oalpha * 0.99 <= alpha.item() <= oalpha * (1 + 1e-9)


def test_barrier_unprojected_parity(abd, ctx):
    S = sg.near_contact_cubes(8, n=3)
    P = sg.default_params()
    sc = abd.Scene(S)
    x = oracle.vertex_map(S, _state(S, 3))
    pt, ee = oracle.candidates(S, x, None, P["dhat"])
    keys = oracle.off_keys(S, pt, ee)
    r = oracle.barrier(S, x, pt, ee, P, keys, project=False)
    e, g, D, O = ctx.barrier_grad_hess(sc, P, _dev(x), _dev(pt, torch.int32), _dev(ee, torch.int32),
                                       _dev(keys, torch.int32), project=False)
    sc_ = np.abs(r["diag"]).max()
    np.testing.assert_allclose(D.cpu().numpy(), r["diag"], rtol=0, atol=1e-10 * sc_)
    np.testing.assert_allclose(O.cpu().numpy(), r["off"], rtol=0, atol=1e-10 * sc_)


def test_barrier_energy_parity(abd, ctx):
    for name, S, P in SCENES:
        sc = abd.Scene(S)
        x = oracle.vertex_map(S, _state(S, 21))
        pt, ee = oracle.candidates(S, x, None, P["dhat"])
        e = ctx.barrier_energy(sc, P, _dev(x), _dev(pt, torch.int32), _dev(ee, torch.int32)).item()
        oe = oracle.barrier_energy(S, x, pt, ee, P)
        assert e == pytest.approx(oe, rel=1e-12, abs=1e-300)


# --------------------------------------------------------- a10 CCD ----

@pytest.mark.parametrize("name,S,P", SCENES, ids=[s[0] for s in SCENES])
def test_ccd_window(abd, ctx, name, S, P):
    sc = abd.Scene(S)
    q0 = _state(S, 31)
    q1 = sg.random_state(S, 32, rot_angle=3e-3, shift=3e-3)
    x0, x1 = oracle.vertex_map(S, q0), oracle.vertex_map(S, q1)
    pt, ee = oracle.candidates(S, x0, x1, P["dhat"])
    tp, te, alpha = ctx.ccd_max_step(sc, P, _dev(x0), _dev(x1 - x0), _dev(pt, torch.int32), _dev(ee, torch.int32))
    otp, ote, oalpha = oracle.ccd(S, x0, x1 - x0, pt, ee, P)
    for t, ot in ((tp.cpu().numpy(), otp), (te.cpu().numpy(), ote)):
        assert np.all(t <= ot * (1 + 1e-9))
        assert np.all(t >= 0.99 * ot)
    assert oalpha * 0.99 <= alpha.item() <= oalpha * (1 + 1e-9)


def test_ccd_grid_queue_and_bound_only_agree(abd, ctx, monkeypatch):
    # the CCD kernel gives each lane its first pair by thread index and the
    # pairs beyond the grid through a work counter; a grid of one block (256
    # lanes) sends almost every pair through the counter.  Per-pair times
    # and the bound are bit-identical either way, and the bound alone (no
    # per-pair output) equals the bound with it.
    S, P = sg.icosphere_box(n_side=3, n_layers=2)
    sc = abd.Scene(S)
    q0 = S["q0"].copy()
    q1 = q0.copy()
    q1[1:, 1] -= 0.4  # (through the lower layer and the floor: a bound below 1)
    q1[1:, 0] += 0.004
    x0, x1 = oracle.vertex_map(S, q0), oracle.vertex_map(S, q1)
    pt, ee = oracle.candidates(S, x0, x1, P["dhat"])
    assert len(pt) + len(ee) > 4 * 256
    args = (sc, P, _dev(x0), _dev(x1 - x0), _dev(pt, torch.int32), _dev(ee, torch.int32))
    monkeypatch.delenv("ABD_CCD_MAX_BLOCKS", raising=False)
    tp, te, a = ctx.ccd_max_step(*args)
    _, _, a_only = ctx.ccd_max_step(*args, per_pair=False)
    monkeypatch.setenv("ABD_CCD_MAX_BLOCKS", "1")
    tp1, te1, a1 = ctx.ccd_max_step(*args)
    _, _, a1_only = ctx.ccd_max_step(*args, per_pair=False)
    monkeypatch.delenv("ABD_CCD_MAX_BLOCKS", raising=False)
    np.testing.assert_array_equal(tp.cpu().numpy(), tp1.cpu().numpy())
    np.testing.assert_array_equal(te.cpu().numpy(), te1.cpu().numpy())
    assert a.item() == a1.item() == a_only.item() == a1_only.item()
    otp, ote, oalpha = oracle.ccd(S, x0, x1 - x0, pt, ee, P)
    assert oalpha < 1.0
    assert oalpha * 0.99 <= a.item() <= oalpha * (1 + 1e-9)


# --------------------------------------------------- a8 body terms ----

def test_orthogonality_inertia_parity(abd, ctx):
    S, P = sg.icosphere_box(n_side=3, n_layers=2)
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    _, vol = oracle.mass_properties(S)
    B = oracle.Body(S)
    q = sg.random_state(S, 41, rot_angle=0.3, stretch=0.05, shift=0.01)
    qt = sg.random_state(S, 42, rot_angle=0.3, stretch=0.05, shift=0.01)
    for project in (0, 1):
        e, g, D = ctx.orthogonality(sc, P, _dev(q), P["dt"] ** 2, project=bool(project))
        oe, og, oD = oracle.orthogonality(S, vol, q, P, project=bool(project))
        assert e.item() == pytest.approx(oe, rel=1e-12)
        np.testing.assert_allclose(g.cpu().numpy(), og, rtol=0, atol=1e-12 * np.abs(og).max())
        np.testing.assert_allclose(D.cpu().numpy(), oD, rtol=0, atol=1e-11 * np.abs(oD).max())
    e, g, D = ctx.inertia(sc, _dev(q), _dev(qt))
    oe, og, oD = oracle.inertia(S, B.M, q, qt)
    assert e.item() == pytest.approx(oe, rel=1e-12)
    np.testing.assert_allclose(g.cpu().numpy(), og, rtol=0, atol=1e-12 * np.abs(og).max())
    np.testing.assert_allclose(D.cpu().numpy(), oD, rtol=0, atol=1e-12 * np.abs(oD).max())
    qd = sg.random_state(S, 43, rot_angle=0.1) - S["q0"]
    qt2 = ctx.q_tilde(sc, P, _dev(q), _dev(qd)).cpu().numpy()
    np.testing.assert_allclose(qt2, oracle.q_tilde(S, q, qd, P), rtol=0, atol=1e-15)


def test_orthogonality_projection_deformed(abd, ctx):
    # projected orthogonality Hessians far from rotations: singular values
    # below 1/sqrt(3) (negative stretch modes), repeated singular values,
    # exact rotations (zero twist modes), reflections, and a nearly singular
    # A, against the oracle's numerical eigen-projection
    S, P = sg.icosphere_box(n_side=3, n_layers=2)
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    _, vol = oracle.mass_properties(S)
    rng = np.random.default_rng(5)
    sigmas = [(0.3, 1.0, 1.5), (0.5, 0.5, 1.2), (1.0, 1.0, 1.0), (0.55, 0.6, 0.58), (1e-5, 1.0, 1.0),
              (0.9, 1.1, -1.0), (2.0, 2.0, 2.0), (0.98, 1.01, 1.02)]
    q = S["q0"].copy()
    free = np.flatnonzero(S["body_fixed"] == 0)
    for n, b in enumerate(free):
        Q1, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        Q2, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        q[b, 3:] = (Q1 @ np.diag(sigmas[n % len(sigmas)]) @ Q2.T).ravel()
    e, g, D = ctx.orthogonality(sc, P, _dev(q), P["dt"] ** 2, project=True)
    oe, og, oD = oracle.orthogonality(S, vol, q, P, project=True)
    assert e.item() == pytest.approx(oe, rel=1e-12)
    Dg = D.cpu().numpy()
    for b in free:
        ref = oD[b]
        np.testing.assert_allclose(Dg[b], ref, rtol=0, atol=1e-11 * np.abs(ref).max())


# ------------------------------------------------------ a9 PCG solve ----

@pytest.mark.parametrize("name,S,P", SCENES[:3] + SCENES[4:], ids=[s[0] for s in SCENES[:3] + SCENES[4:]])
def test_pcg_matches_direct_solve(abd, ctx, name, S, P):
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    B = oracle.Body(S)
    q = _state(S, 51)
    qt = q.copy()
    qt[:, :3] += P["dt"] ** 2 * np.array(P["gravity"])
    qt[S["body_fixed"] != 0] = q[S["body_fixed"] != 0]
    gh = oracle.grad_hess(S, B, q, qt, P)
    p_ref = oracle.solve(S, gh["diag"], gh["off"], gh["keys"], -gh["grad"])
    p, its = ctx.pcg_solve(sc, _dev(gh["diag"]), _dev(gh["off"].reshape(-1, 144) if len(gh["keys"]) else
                                                     np.zeros((1, 144))),
                           _dev(gh["keys"], torch.int32), _dev(-gh["grad"]), rtol=1e-14, max_iter=20000)
    p = p.cpu().numpy()
    assert np.abs(p - p_ref).max() <= 1e-8 * np.abs(p_ref).max()


@pytest.mark.parametrize("form", ["two_kernel", "one_kernel"])
@pytest.mark.parametrize("rtol", [1e-6, 1e-13])
def test_pcg_forms_match_direct_solve(abd, ctx, form, rtol, monkeypatch):
    # both iteration forms (the one-kernel form is followed by the check on
    # a fresh residual; ABD_PCG_CG=0 selects the two-kernel form alone) meet
    # the tolerance on the true residual, against the oracle's direct solve
    if form == "two_kernel":
        monkeypatch.setenv("ABD_PCG_CG", "0")
    else:
        monkeypatch.delenv("ABD_PCG_CG", raising=False)
    name, S, P = SCENES[0]
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    B = oracle.Body(S)
    q = _state(S, 52)
    qt = q.copy()
    qt[:, :3] += P["dt"] ** 2 * np.array(P["gravity"])
    qt[S["body_fixed"] != 0] = q[S["body_fixed"] != 0]
    gh = oracle.grad_hess(S, B, q, qt, P)
    p_ref = oracle.solve(S, gh["diag"], gh["off"], gh["keys"], -gh["grad"])
    p, its = ctx.pcg_solve(sc, _dev(gh["diag"]), _dev(gh["off"].reshape(-1, 144)), _dev(gh["keys"], torch.int32),
                           _dev(-gh["grad"]), rtol=rtol, max_iter=20000)
    assert its > 0
    p = p.cpu().numpy()
    free = S["body_fixed"] == 0
    A = oracle.assemble(S, gh["diag"], gh["off"], gh["keys"])[0]
    b = -gh["grad"][free].ravel()
    res = A @ p[free].ravel() - b
    if rtol >= 1e-8:  # (at tighter tolerances the residual's own rounding dominates)
        assert np.linalg.norm(res) <= rtol * np.linalg.norm(b) * 1.01
    else:
        assert np.abs(p - p_ref).max() <= 1e-8 * np.abs(p_ref).max()


# ------------------------------------------------- a11/a12 Newton ----

@pytest.mark.parametrize("name,S,P", SCENES[:3] + SCENES[4:], ids=[s[0] for s in SCENES[:3] + SCENES[4:]])
def test_newton_step_parity(abd, ctx, name, S, P):
    P = dict(P, pcg_rtol=1e-14, max_pcg=20000)
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    B = oracle.Body(S)
    q = _state(S, 61)
    qd = np.zeros_like(q)
    qd[S["body_fixed"] == 0, 1] = -0.05
    qt = oracle.q_tilde(S, q, qd, P)
    qn_ref, conv_ref, info = oracle.newton_iteration(S, B, q, qt, P)
    qg = _dev(q)
    st = ctx.newton_step(sc, P, qg, _dev(qt))
    assert bool(st["converged"]) == conv_ref
    d_ref = info["p"]
    dq = qg.cpu().numpy() - q
    if not conv_ref:
        assert st["alpha"] == pytest.approx(info["alpha"], rel=1e-2)
        # Newton step q_new - q within 1e-8 of the oracle's
        ref = qn_ref - q
        assert np.abs(dq - ref).max() <= 1e-8 * np.abs(ref).max()
    assert st["n_active_pt"] + st["n_active_ee"] == info["n_active"]
    assert st["disp"] == pytest.approx(info["disp"], rel=1e-6)


def test_time_steps_three_cubes_trajectory(abd, ctx):
    S, P = sg.three_cubes()
    P = dict(P, pcg_rtol=1e-13, max_pcg=20000)
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    B = oracle.Body(S)
    q, qd = S["q0"].copy(), S["qd0"].copy()
    qg, qdg = _dev(q), _dev(qd)
    for step in range(25):
        q, qd, its = oracle.time_step(S, B, q, qd, P)
        st = ctx.time_step(sc, P, qg, qdg)
        assert st["converged"] == 1
        # trajectories agree while contacts form (per-step tolerance loose:
        # different Newton paths converge to the same minimiser within tol)
        np.testing.assert_allclose(qg.cpu().numpy(), q, rtol=0, atol=1e-6)


def test_pcg_graph_replays_match_eager(abd, ctx):
    """The PCG iterations run from a captured graph; every replay (with eager
    library work and synchronisations in between) must equal the eagerly
    launched kernels bit for bit, and the direct solve to 1e-8."""
    import os
    S = sg.near_contact_cubes(1, n=4)
    P = dict(sg.default_params())
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    B = oracle.Body(S)
    q = _state(S, 71)
    qt = q.copy()
    qt[:, :3] += P["dt"] ** 2 * np.array(P["gravity"])
    qt[S["body_fixed"] != 0] = q[S["body_fixed"] != 0]
    gh = oracle.grad_hess(S, B, q, qt, P)
    args = (_dev(gh["diag"]), _dev(gh["off"]), _dev(gh["keys"], torch.int32), _dev(-gh["grad"]))
    p_ref = oracle.solve(S, gh["diag"], gh["off"], gh["keys"], -gh["grad"])
    os.environ["ABD_PCG_GRAPH"] = "0"
    try:
        p_eager, it_eager = ctx.pcg_solve(sc, *args, rtol=1e-14, max_iter=20000)
    finally:
        del os.environ["ABD_PCG_GRAPH"]
    p_eager = p_eager.cpu().numpy()
    assert np.abs(p_eager - p_ref).max() <= 1e-8 * np.abs(p_ref).max()
    x = _dev(oracle.vertex_map(S, q))
    for rep in range(4):
        p, it = ctx.pcg_solve(sc, *args, rtol=1e-14, max_iter=20000)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(p.cpu().numpy(), p_eager)
        assert it == it_eager
        ctx.vertex_map(sc, _dev(q))            # eager work between replays
        ctx.candidates(sc, x, None, P["dhat"])


def test_pcg_tolerance_change_recaptures(abd, ctx):
    """Two solves of one system with different tolerances in a row: the
    captured iterations must follow each call's tolerance."""
    S = sg.near_contact_cubes(2, n=4)
    P = dict(sg.default_params())
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    B = oracle.Body(S)
    q = _state(S, 72)
    qt = q.copy()
    qt[:, :3] += P["dt"] ** 2 * np.array(P["gravity"])
    qt[S["body_fixed"] != 0] = q[S["body_fixed"] != 0]
    gh = oracle.grad_hess(S, B, q, qt, P)
    args = (_dev(gh["diag"]), _dev(gh["off"]), _dev(gh["keys"], torch.int32), _dev(-gh["grad"]))
    p_ref = oracle.solve(S, gh["diag"], gh["off"], gh["keys"], -gh["grad"])
    _, it_loose = ctx.pcg_solve(sc, *args, rtol=1e-2, max_iter=20000)
    p, it_tight = ctx.pcg_solve(sc, *args, rtol=1e-14, max_iter=20000)
    assert it_tight > it_loose
    assert np.abs(p.cpu().numpy() - p_ref).max() <= 1e-8 * np.abs(p_ref).max()
    _, it_loose2 = ctx.pcg_solve(sc, *args, rtol=1e-2, max_iter=20000)
    assert it_loose2 == it_loose


@pytest.mark.parametrize("name,S,P", SCENES, ids=[s[0] for s in SCENES])
def test_candidates_within_sweep_equal_full_broad_phase(abd, ctx, name, S, P):
    """Static candidates taken from a sweep's candidates equal the full broad
    phase at points of the segment (the Newton loop relies on it)."""
    sc = abd.Scene(S)
    q0 = _state(S, 41)
    q1 = sg.random_state(S, 42, rot_angle=3e-3, shift=3e-3)
    x0, x1 = oracle.vertex_map(S, q0), oracle.vertex_map(S, q1)
    spt, see = ctx.candidates(sc, _dev(x0), _dev(x1), P["dhat"])
    for a in (0.0, 0.3, 0.77, 1.0):
        xa = oracle.vertex_map(S, q0 + a * (q1 - q0))
        fpt, fee = ctx.candidates(sc, _dev(xa), None, P["dhat"])
        wpt, wee = ctx.candidates_within(sc, _dev(xa), spt, see, P["dhat"])
        np.testing.assert_array_equal(wpt.cpu().numpy(), fpt.cpu().numpy())
        np.testing.assert_array_equal(wee.cpu().numpy(), fee.cpu().numpy())


def test_pcg_initial_guess(abd, ctx):
    """PCG from an initial guess: the solution itself stops at once; any
    other guess reaches the direct solution; the tolerance is relative to
    the right-hand side, not to the initial residual."""
    S = sg.near_contact_cubes(3, n=4)
    P = dict(sg.default_params())
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    B = oracle.Body(S)
    q = _state(S, 73)
    qt = q.copy()
    qt[:, :3] += P["dt"] ** 2 * np.array(P["gravity"])
    qt[S["body_fixed"] != 0] = q[S["body_fixed"] != 0]
    gh = oracle.grad_hess(S, B, q, qt, P)
    args = (_dev(gh["diag"]), _dev(gh["off"]), _dev(gh["keys"], torch.int32), _dev(-gh["grad"]))
    p_ref = oracle.solve(S, gh["diag"], gh["off"], gh["keys"], -gh["grad"])
    _, it_sol = ctx.pcg_solve(sc, *args, rtol=1e-6, max_iter=20000, x0=_dev(p_ref))
    assert it_sol == 0
    x0 = np.random.default_rng(5).normal(size=p_ref.shape) * np.abs(p_ref).max()
    x0[S["body_fixed"] != 0] = 0.0
    p, it = ctx.pcg_solve(sc, *args, rtol=1e-14, max_iter=20000, x0=_dev(x0))
    assert it > 0
    assert np.abs(p.cpu().numpy() - p_ref).max() <= 1e-8 * np.abs(p_ref).max()

"""The three-level i-AABB tree (sec. 4.2, Fig. iBVH) against the single
i-AABB: the same candidate pairs in the same order (arrays equal element
by element), the set equal to the oracle's box predicate, and fewer
primitive-pair box tests where contact is entangled.

Workloads: the 64 interlocked links in contact (static, and swept over one
step of their initial velocities), the box drop's bottom layers at landing,
the three-cube scene (lists shorter than one 64-chunk: the tree has one
leaf) and a triangle soup (many small bodies).  Each at two tile heights,
since tiles must stay inside one row leaf."""
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


def _sorted(a):
    a = np.asarray(a, dtype=np.int64).reshape(-1, 2)
    return a[np.lexsort((a[:, 1], a[:, 0]))] if len(a) else a


def _run(ctx, sc, x0, x1, inflate, levels, trows):
    ctx.tune_set(dict(cull_levels=levels, tile_rows=trows))
    ctx.profile(2, True)
    pt, ee = ctx.candidates(sc, x0, x1, inflate)
    tests = ctx.profile_query("box_tests")["units"]
    flat = ctx.profile_query("box_tests_single_level")["units"]
    ctx.profile(False, True)
    return pt.cpu().numpy(), ee.cpu().numpy(), tests, flat


def _compare(ctx, sc, S, x0, x1, inflate, with_oracle=True):
    """Tree and single level at tile heights 8 and 64: equal arrays; the
    oracle's sets; the box-test counts (tree, single level)."""
    x0g = _dev(x0)
    x1g = None if x1 is None else _dev(x1)
    ref = None
    counts = {}
    for trows in (8, 64):
        for levels in (1, 3):
            pt, ee, tests, flat = _run(ctx, sc, x0g, x1g, inflate, levels, trows)
            counts[levels] = (tests, flat)
            if ref is None:
                ref = (pt, ee)
            else:
                np.testing.assert_array_equal(pt, ref[0])
                np.testing.assert_array_equal(ee, ref[1])
        assert counts[1][0] == counts[1][1] == counts[3][1]
        assert counts[3][0] <= counts[1][0]
    ctx.tune_set(dict(cull_levels=1, tile_rows=16))
    if with_oracle:
        opt, oee = oracle.candidates(S, x0, x1, inflate)
        np.testing.assert_array_equal(_sorted(ref[0]), opt)
        np.testing.assert_array_equal(_sorted(ref[1]), oee)
    return len(ref[0]) + len(ref[1]), counts[3][0], counts[1][0]


def test_tree_on_interlocked_links(abd, ctx):
    S, P = sg.torus_chains()
    sc = abd.Scene(S)
    q = sg.torus_chains_contact(S, 8)
    x = oracle.vertex_map(S, q)
    n, tree, flat = _compare(ctx, sc, S, x, None, P["dhat"], with_oracle=False)
    assert n > 0
    x1 = oracle.vertex_map(S, q + P["dt"] * S["qd0"])
    n, tree, flat = _compare(ctx, sc, S, x, x1, P["dhat"])
    assert n > 10000
    # entangled links: the leaves of one link's culled lists meet only
    # part of the other's
    assert tree < 0.8 * flat, (tree, flat)


def test_tree_on_box_drop_and_small_scenes(abd, ctx):
    S, P = sg.icosphere_box(n_layers=2)
    S = sg.landed(S, seed=7, dhat=P["dhat"])
    sc = abd.Scene(S)
    x = oracle.vertex_map(S, S["q0"])
    x1 = oracle.vertex_map(S, S["q0"] + P["dt"] * S["qd0"])
    n, _, _ = _compare(ctx, sc, S, x, x1, P["dhat"])
    assert n > 0
    for S, inflate in ((sg.three_cubes()[0], 2e-2), (sg.triangle_soup(3), 2e-3)):
        sc = abd.Scene(S)
        x = oracle.vertex_map(S, S["q0"])
        n, _, _ = _compare(ctx, sc, S, x, None, inflate)
        assert n > 0

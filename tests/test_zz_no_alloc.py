"""The allocation-free barrier-energy entry point against abd_barrier_energy
(same kernels and summation order: bit for bit) and the oracle (1e-12
relative), called through the C ABI twice in a row, the second call with a
smaller input (the scratch array keeps the first call's contents), and its
capacity check."""
import ctypes

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


def _dev(a, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda:0")


def _case(S, P):
    x = oracle.vertex_map(S, S["q0"])
    pt, ee = oracle.candidates(S, x, None, P["dhat"])
    return x, pt, ee


def test_barrier_energy_noalloc_matches(abd):
    ctx = abd.Context(0)
    # first call: 416k pairs of the FCC packing (two-pass reduction);
    # second: the box's resting bottom layer, far fewer pairs (one pass)
    cases = [sg.icosphere_fcc(), sg.icosphere_resting_layer()]
    sizes = []
    for S, P in cases:
        sc = abd.Scene(S)
        x, pt, ee = _case(S, P)
        xg, ptg, eeg = _dev(x), _dev(pt, torch.int32), _dev(ee, torch.int32)
        ref = ctx.barrier_energy(sc, P, xg, ptg, eeg).item()
        got = ctx.barrier_energy_noalloc(sc, P, xg, ptg, eeg).item()
        assert got == ref
        ora = oracle.barrier_energy(S, x, pt, ee, P)
        assert got == pytest.approx(ora, rel=1e-12)
        assert got > 0.0
        sizes.append(len(pt) + len(ee))
    assert sizes[0] > 16 * 1024 > sizes[1] > 0
    # accumulation into the caller's value, as abd_barrier_energy
    S, P = cases[1]
    sc = abd.Scene(S)
    x, pt, ee = _case(S, P)
    e = torch.full((1,), 2.5, dtype=torch.float64, device="cuda:0")
    ctx.barrier_energy_noalloc(sc, P, _dev(x), _dev(pt, torch.int32), _dev(ee, torch.int32), energy=e)
    ref = ctx.barrier_energy(sc, P, _dev(x), _dev(pt, torch.int32), _dev(ee, torch.int32)).item()
    assert e.item() == 2.5 + ref


def test_barrier_energy_noalloc_capacity(abd):
    # more pairs than the scratch holds: refused on the host before any launch
    ctx = abd.Context(0)
    S, P = sg.three_cubes()
    sc = abd.Scene(S)
    x = _dev(oracle.vertex_map(S, S["q0"]))
    pairs = torch.zeros((1, 2), dtype=torch.int32, device="cuda:0")
    e = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    prm = abd.make_params(P)
    rc = ctx.L.abd_barrier_energy_noalloc(ctx.h, ctypes.byref(sc.c), ctypes.byref(prm), abd._ptr(x),
                                          abd._ptr(pairs), (1 << 20) + 1, abd._ptr(pairs), 0, abd._ptr(e),
                                          abd._stream())
    assert rc == -2
    assert b"scratch capacity" in ctx.L.abd_last_error(ctx.h)
    assert e.item() == 0.0

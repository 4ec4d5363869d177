"""GPU parity of the alternative rigidity potentials (ARAP and neo-Hookean,
sec. 3.2) against the oracle: per-body energies, gradients and Hessian
blocks (unprojected and PSD-projected) on strongly deformed bodies, the
energy-only path, and Newton steps of a near-contact cube stack with each
potential.  The GPU forms everything from A's signed singular values
(closed-form eigensystems); the oracle from the polar decomposition's
differential and the neo-Hookean closed forms."""
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


def _deformed_state(S, seed, eps):
    rng = np.random.default_rng(seed)
    q = S["q0"].copy()
    for b in np.flatnonzero(S["body_fixed"] == 0):
        Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        Q *= np.sign(np.linalg.det(Q))
        q[b, 3:] = (Q @ (np.eye(3) + eps * rng.normal(size=(3, 3)))).reshape(9)
    return q


@pytest.mark.parametrize("rigidity", [1, 2])
def test_rigidity_terms_parity(abd, ctx, rigidity):
    S, P = sg.icosphere_box(n_side=3, n_layers=2)
    P = dict(P, rigidity=rigidity)
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    _, vol = oracle.mass_properties(S)
    for seed, eps in ((1, 0.05), (2, 0.3)):
        q = _deformed_state(S, seed, eps)
        for project in (False, True):
            e, g, D = ctx.orthogonality(sc, P, _dev(q), P["dt"] ** 2, project=project)
            oe, og, oD = oracle.rigidity(S, vol, q, P, project=project)
            assert e.item() == pytest.approx(oe, rel=1e-12)
            np.testing.assert_allclose(g.cpu().numpy(), og, rtol=0, atol=1e-12 * np.abs(og).max())
            Dg = D.cpu().numpy()
            for b in np.flatnonzero(S["body_fixed"] == 0):
                np.testing.assert_allclose(Dg[b], oD[b], rtol=0, atol=1e-10 * np.abs(oD[b]).max())
        # energy-only path
        eo = ctx.orthogonality(sc, P, _dev(q), P["dt"] ** 2, project=False, hessian=False)[0].item()
        assert eo == pytest.approx(oe, rel=1e-12)


@pytest.mark.parametrize("rigidity", [1, 2])
def test_newton_step_with_rigidity(abd, ctx, rigidity):
    S = sg.near_contact_cubes(3, n=4)
    P = dict(sg.default_params(kappa_b=80.0), rigidity=rigidity, pcg_rtol=1e-14, max_pcg=20000)
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    B = oracle.Body(S)
    q = _deformed_state(S, 5, 1e-3)
    qd = np.zeros_like(q)
    qd[S["body_fixed"] == 0, 1] = -0.05
    qt = oracle.q_tilde(S, q, qd, P)
    qn_ref, conv, info = oracle.newton_iteration(S, B, q, qt, P)
    assert not conv
    qg = _dev(q)
    st = ctx.newton_step(sc, P, qg, _dev(qt))
    ref = qn_ref - q
    err = np.abs(qg.cpu().numpy() - q - ref).max() / np.abs(ref).max()
    assert err <= 1e-8, err

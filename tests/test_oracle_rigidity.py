"""Pins of the oracle's alternative rigidity potentials (ARAP and
neo-Hookean, sec. 3.2's alternatives to the orthogonality potential):
zero energy and force on rotations, closed forms on A = s I, gradients and
Hessians against central differences, the Hessians' spectra at a rotation
(ARAP: 2 on the six stretch modes, 0 on the three twists; neo-Hookean at
I: 2 mu on the five traceless symmetric modes, 2 mu + 3 lambda on the
dilation, 0 on the twists), and the scaled per-body assembly."""
import math

import numpy as np
import pytest

import oracle
import scenegen as sg


def _rot(rng):
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    return Q * np.sign(np.linalg.det(Q))


def _deformed(rng, eps=0.2):
    return _rot(rng) @ (np.eye(3) + eps * rng.normal(size=(3, 3)))


def _fd_grad(f, A, h=1e-6):
    g = np.zeros(9)
    for k in range(9):
        d = np.zeros(9)
        d[k] = h
        g[k] = (f(A + d.reshape(3, 3)) - f(A - d.reshape(3, 3))) / (2 * h)
    return g


def _fd_hess(gf, A, h=1e-6):
    H = np.zeros((9, 9))
    for k in range(9):
        d = np.zeros(9)
        d[k] = h
        H[:, k] = (gf(A + d.reshape(3, 3)) - gf(A - d.reshape(3, 3))) / (2 * h)
    return H


KINDS = {"arap": lambda A: oracle.arap_body(A), "nh": lambda A: oracle.neo_hookean_body(A, 1.0, 1.0)}


@pytest.mark.parametrize("kind", list(KINDS))
def test_zero_on_rotations(kind):
    rng = np.random.default_rng(1)
    for _ in range(5):
        e, g, H = KINDS[kind](_rot(rng))
        assert abs(e) < 1e-13 and np.abs(g).max() < 1e-12


def test_closed_forms_on_scaling():
    for s in (0.5, 0.9, 1.0, 1.3, 2.0):
        e, g, _ = oracle.arap_body(s * np.eye(3))
        assert e == pytest.approx(3 * (s - 1) ** 2, abs=1e-14)
        np.testing.assert_allclose(g.reshape(3, 3), 2 * (s - 1) * np.eye(3), atol=1e-14)
        e, g, _ = oracle.neo_hookean_body(s * np.eye(3), 1.0, 1.0)
        ls = math.log(s)
        assert e == pytest.approx(0.5 * (3 * s * s - 3) - 3 * ls + 0.5 * (3 * ls) ** 2, rel=1e-13, abs=1e-14)
        np.testing.assert_allclose(g.reshape(3, 3), (s - 1 / s + 3 * ls / s) * np.eye(3), atol=1e-13)
    assert oracle.neo_hookean_body(np.diag([1.0, 1.0, -1.0]), 1.0, 1.0)[0] == np.inf


@pytest.mark.parametrize("kind", list(KINDS))
def test_derivatives_by_finite_differences(kind):
    rng = np.random.default_rng(2)
    f = KINDS[kind]
    for _ in range(6):
        A = _deformed(rng)
        e, g, H = f(A)
        np.testing.assert_allclose(g, _fd_grad(lambda X: f(X)[0], A), rtol=0, atol=1e-7 * max(1, np.abs(g).max()))
        np.testing.assert_allclose(H, _fd_hess(lambda X: f(X)[1], A), rtol=0, atol=1e-6 * np.abs(H).max())


def test_spectra_at_rest():
    rng = np.random.default_rng(3)
    R = _rot(rng)
    lam = np.sort(np.linalg.eigvalsh(oracle.arap_body(R)[2]))
    np.testing.assert_allclose(lam, [0, 0, 0, 2, 2, 2, 2, 2, 2], atol=1e-12)
    mu, la = 1.0, 1.0
    lam = np.sort(np.linalg.eigvalsh(oracle.neo_hookean_body(np.eye(3), mu, la)[2]))
    np.testing.assert_allclose(lam, [0, 0, 0] + [2 * mu] * 5 + [2 * mu + 3 * la], atol=1e-12)


@pytest.mark.parametrize("rigidity", [1, 2])
def test_assembly_scaled_and_projected(rigidity):
    S, P = sg.icosphere_box(n_side=2, n_layers=1)
    P = dict(P, rigidity=rigidity)
    _, vol = oracle.mass_properties(S)
    rng = np.random.default_rng(4)
    q = S["q0"].copy()
    free = np.flatnonzero(S["body_fixed"] == 0)
    for b in free:
        q[b, 3:] = _deformed(rng, 0.3).reshape(9)
    e, g, D = oracle.rigidity(S, vol, q, P, project=False)
    ep, gp, Dp = oracle.rigidity(S, vol, q, P, project=True)
    w = P["dt"] ** 2
    tot = 0.0
    for b in free:
        eb, gb, Hb = KINDS["arap" if rigidity == 1 else "nh"](q[b, 3:].reshape(3, 3))
        c = P["kappa_o"] * vol[b] * w
        tot += c * eb
        np.testing.assert_allclose(g[b, 3:], c * gb, rtol=1e-14, atol=0)
        Hf = D[b].reshape(12, 12)
        np.testing.assert_allclose(Hf[3:, 3:], c * Hb, rtol=1e-14, atol=0)
        assert not Hf[:3].any() and not Hf[:, :3].any()
        Hp = Dp[b].reshape(12, 12)[3:, 3:]
        assert np.linalg.eigvalsh(Hp).min() >= -1e-9 * np.abs(Hp).max()
        lam, V = np.linalg.eigh(Hf[3:, 3:])
        np.testing.assert_allclose(Hp, (V * np.maximum(lam, 0)) @ V.T, rtol=0, atol=1e-9 * np.abs(Hp).max())
    assert e == pytest.approx(tot, rel=1e-13) and ep == e

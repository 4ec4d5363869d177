"""Pins of the oracle's adaptive barrier stiffness (IPC's rule, read for
the paper's kappa; see barrier_stiffness_init in the oracle).

The initial value against a closed form: a right-corner tetrahedron (legs
a, density rho, corner at the body origin) resting with its x-z face a
height d over a large fixed triangle, at rest, so that the three vertices of
that face are the only active pairs.  With g = (0, g_y, 0):
  g_E = M (q - q~) = -dt^2 f, f = (m g, g_i mom_j) (mom = m (a/4, a/4, a/4)),
  g_B = B'(d) (3 e_{p_y} + sum_j s_j e_{A_yj}), s = sum of the face's body
        points = (a, 0, a),
so kappa = -(g_E . g_B) / |g_B|^2 = dt^2 g_y m (3 + a^2/2) / (B'(d) (9 + 2 a^2))
with B(d) = -(d - dhat)^2 ln(d / dhat).  The doubling rule on scripted
distances; a drop onto the ground that doubles kappa while approaching."""
import math

import numpy as np
import pytest

import oracle
import scenegen as sg


def _bprime(d, dhat):
    return -2.0 * (d - dhat) * math.log(d / dhat) - (d - dhat) ** 2 / d


@pytest.mark.parametrize("a,d", [(0.5, 3e-4), (0.2, 7e-4)])
def test_initial_kappa_closed_form(a, d):
    S, P = sg.tet_over_ground(a=a, height=d)
    P = dict(P, kappa_b=1e-30, kappa_max=1e30)
    B = oracle.Body(S)
    q = S["q0"]
    qt = oracle.q_tilde(S, q, S["qd0"], P)
    kappa, d2 = oracle.barrier_stiffness_init(S, B, q, qt, P)
    m = 1000.0 * a ** 3 / 6.0
    gy = P["gravity"][1]
    ref = P["dt"] ** 2 * gy * m * (3.0 + a * a / 2.0) / (_bprime(d, P["dhat"]) * (9.0 + 2.0 * a * a))
    assert ref > 0
    assert kappa == pytest.approx(ref, rel=1e-10)
    assert math.sqrt(d2) == pytest.approx(d, rel=1e-9)
    # the clamp
    lo = oracle.barrier_stiffness_init(S, B, q, qt, dict(P, kappa_b=2 * ref))[0]
    hi = oracle.barrier_stiffness_init(S, B, q, qt, dict(P, kappa_max=0.5 * ref))[0]
    assert lo == 2 * ref and hi == 0.5 * ref


def test_initial_kappa_without_contact_is_the_floor():
    S, P = sg.tet_over_ground(height=0.1)
    B = oracle.Body(S)
    qt = oracle.q_tilde(S, S["q0"], S["qd0"], P)
    kappa, d2 = oracle.barrier_stiffness_init(S, B, S["q0"], qt, P)
    assert kappa == P["kappa_b"] and d2 == np.inf


def test_doubling_rule():
    P = dict(kappa_eps_d=1e-5, kappa_max=100.0)
    up = oracle.barrier_stiffness_update
    assert up(10.0, 0.5e-10, 0.9e-10, P) == 20.0           # below eps and approaching
    assert up(60.0, 0.5e-10, 0.9e-10, P) == 100.0          # capped
    assert up(10.0, 0.9e-10, 0.5e-10, P) == 10.0           # receding
    assert up(10.0, 2e-10, 3e-10, P) == 10.0               # above eps (eps^2 = 1e-10)
    assert up(10.0, 0.5e-10, 0.5e-10, P) == 10.0           # equal: not approaching


def test_drop_raises_kappa_while_approaching():
    # the tetrahedron hits the ground at 0.5 m/s from 2 mm; with eps_d = dhat
    # every iteration that brings the face closer within dhat doubles kappa;
    # the contact stays open
    S, P = sg.tet_over_ground(height=2e-3, v0=0.5)
    P = dict(P, kappa_adaptive=1, kappa_eps_d=P["dhat"])
    B = oracle.Body(S)
    q, qd = S["q0"].copy(), S["qd0"].copy()
    kappas = []
    for _ in range(4):
        log = []
        q, qd, _ = oracle.time_step(S, B, q, qd, P, log=log)
        kappas += [l["kappa_b"] for l in log]
        x = oracle.vertex_map(S, q)
        assert x[3:, 1].min() > 0.0
    assert kappas[0] >= P["kappa_b"]
    assert max(kappas) > kappas[0]
    assert max(kappas) <= P["kappa_max"]
    # an adaptive rollout cannot be differentiated
    with pytest.raises(ValueError):
        oracle.rollout_grad(S, B, S["q0"], S["qd0"], P, 1, np.zeros_like(q), np.zeros_like(q))

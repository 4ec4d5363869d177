"""GPU parity of the adaptive barrier stiffness (IPC's rule for the paper's
kappa; abd_params.kappa_adaptive) against the oracle's.

- The initial value on the tetrahedron resting a height d over a triangle
  (three active point-triangle pairs): the closed form of the oracle's pin,
  the oracle's value, and the GPU's (one time step with eps_d = 0, so no
  doubling), within 1e-12.
- A drop of the tetrahedron at 0.5 m/s from 2 mm with eps_d = dhat (kappa
  doubles while the face approaches): four time steps, states within 1e-7
  and the final kappa equal to the oracle's.
- The box drop's two bottom layers at landing, adaptive with floor 1 and
  eps_d = dhat/4 (the start value from the gradient balance, and doublings
  as spheres approach): three steps within 1e-6 of the oracle's trajectory
  and the same kappa.
- A batch of 16 drop scenes at landing: per-scene kappa in one batch equal,
  state (vertices within twice the Newton stopping distance) and stiffness
  (1e-6 relative), to each scene run on its own, and different between
  scenes.
- abd_newton_step and the rollouts reject the adaptive flag."""
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


def _bprime(d, dhat):
    return -2.0 * (d - dhat) * math.log(d / dhat) - (d - dhat) ** 2 / d


def test_initial_kappa_resting_tetrahedron(abd, ctx):
    a, d = 0.5, 3e-4
    S, P = sg.tet_over_ground(a=a, height=d)
    P = dict(P, kappa_adaptive=1, kappa_b=1e-6, kappa_max=1e12, kappa_eps_d=0.0)
    m = 1000.0 * a ** 3 / 6.0
    ref = P["dt"] ** 2 * P["gravity"][1] * m * (3 + a * a / 2) / (_bprime(d, P["dhat"]) * (9 + 2 * a * a))
    B = oracle.Body(S)
    qt = oracle.q_tilde(S, S["q0"], S["qd0"], P)
    k_ora, _ = oracle.barrier_stiffness_init(S, B, S["q0"], qt, P)
    assert k_ora == pytest.approx(ref, rel=1e-10)
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    q, qd = _dev(S["q0"]), _dev(S["qd0"])
    ctx.time_step(sc, P, q, qd)
    k = ctx.barrier_stiffness(sc)
    assert k.shape == (1,)
    assert k[0] == pytest.approx(k_ora, rel=1e-12)


def test_tetrahedron_drop_doubles_like_the_oracle(abd, ctx):
    S, P = sg.tet_over_ground(height=2e-3, v0=0.5)
    P = dict(P, kappa_adaptive=1, kappa_eps_d=P["dhat"])
    B = oracle.Body(S)
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    q, qd = S["q0"].copy(), S["qd0"].copy()
    qg, qdg = _dev(q), _dev(qd)
    kappas = []
    for _ in range(4):
        log = []
        q, qd, _ = oracle.time_step(S, B, q, qd, P, log=log)
        kappas.append(log[-1]["kappa_b"])
        ctx.time_step(sc, P, qg, qdg)
        np.testing.assert_allclose(qg.cpu().numpy(), q, rtol=0, atol=1e-7)
        assert ctx.barrier_stiffness(sc)[0] == pytest.approx(kappas[-1], rel=1e-12)
    assert max(kappas) > P["kappa_b"]


def test_box_landing_adaptive_trajectory(abd, ctx):
    S, P = sg.icosphere_box(n_layers=2)
    S = sg.landed(S, seed=7, dhat=P["dhat"])
    # (floor 1: the gradient balance, about 5 here, sets the start value)
    P = dict(P, mu=0.0, kappa_adaptive=1, kappa_b=1.0, kappa_max=7000.0, kappa_eps_d=P["dhat"] / 4,
             newton_tol=1e-6, pcg_rtol=1e-13, max_pcg=20000, max_newton=200)
    B = oracle.Body(S)
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    q, qd = S["q0"].copy(), S["qd0"].copy()
    qg, qdg = _dev(q), _dev(qd)
    doubled = 0
    for _ in range(3):
        log = []
        q, qd, _ = oracle.time_step(S, B, q, qd, P, log=log)
        ks = [l["kappa_b"] for l in log]
        assert ks[0] > P["kappa_b"]
        doubled += sum(b == 2 * a for a, b in zip(ks, ks[1:]))
        ctx.time_step(sc, P, qg, qdg)
        np.testing.assert_allclose(qg.cpu().numpy(), q, rtol=0, atol=1e-6)
        assert ctx.barrier_stiffness(sc)[0] == pytest.approx(ks[-1], rel=1e-9)
    assert doubled >= 2


def test_batched_kappa_per_scene(abd, ctx):
    S, P = sg.batched_drops(n_scenes=16)
    # (the workload's own tolerances: batch and single scenes take the same
    # decisions, so they agree far below them)
    Pf = P
    P = dict(Pf, kappa_adaptive=1, kappa_b=1.0, kappa_max=7000.0, kappa_eps_d=P["dhat"] / 4)
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    q, qd = _dev(S["q0"]), _dev(S["qd0"])
    for _ in range(22):  # (fixed stiffness until the lowest layers land)
        ctx.time_step(sc, Pf, q, qd)
    q0, qd0 = q.clone(), qd.clone()
    for _ in range(2):
        ctx.time_step(sc, P, q, qd)
    kb = ctx.barrier_stiffness(sc)
    assert len(kb) == 16 and len(np.unique(kb)) > 1
    qb = q.cpu().numpy()
    off = S["scene_body_off"]
    for k in range(16):
        Sk = sg.sub_scene(S, k)
        sck = abd.Scene(Sk)
        ctx.body_mass(sck)
        b0, b1 = off[k], off[k + 1]
        qk, qdk = q0[b0:b1].clone(), qd0[b0:b1].clone()
        for _ in range(2):
            ctx.time_step(sck, P, qk, qdk)
        ref = qk.cpu().numpy()
        # (a one-scene run sums a trial's energies in one row, a batch per
        # scene: the line searches compare energies rounded differently, so
        # the two runs may stop Newton at different iterates; each is within
        # about tol_v dt of the minimiser, so vertices agree to twice that)
        bar = 2.0 * (1.0 + P["pcg_rtol"]) * P["newton_tol"] * P["dt"]
        dx = np.abs(oracle.vertex_map(Sk, qb[b0:b1]) - oracle.vertex_map(Sk, ref)).max()
        assert dx <= bar, (k, dx, bar)
        assert ctx.barrier_stiffness(sck)[0] == pytest.approx(kb[k], rel=1e-6)


def test_adaptive_flag_rejected_outside_time_steps(abd, ctx):
    S, P = sg.tet_over_ground()
    P = dict(P, kappa_adaptive=1)
    sc = abd.Scene(S)
    ctx.body_mass(sc)
    q, qd = _dev(S["q0"]), _dev(S["qd0"])
    with pytest.raises(abd.AbdError):
        ctx.newton_step(sc, P, q.clone(), q.clone())
    with pytest.raises(abd.AbdError):
        ctx.rollout_forward(sc, P, q.clone(), qd.clone(), 1)

"""Throughput of the affine-body contact path on one MI355X.

A step is one implicit-Euler time step of the 1000-icosphere box drop
(162,017 vertices, 320,024 triangles, 480,040 edges, 12,000 free DOFs,
FP64): every Newton iteration runs the kinematic map, both candidate
sweeps, the barrier gradient and PSD-projected Hessian with J^T H J
assembly, the body terms, the PCG solve, CCD and the line search.  The
scene is first advanced (untimed) until the spheres have landed, so the
timed steps run in contact.

Printed JSON line: value = contact-pair evaluations per second (active
pairs through the barrier kernels plus pairs through CCD, summed over
every Newton iteration of the timed steps, divided by the timed
wall-clock), plus Newton iterations per second, the roofline position of
the dominant kernel (HIP events inside the library) and the CPU oracle's
rate on a bounded sample.

With --workload batched the step is one time step of 256 independent
drop scenes (26,914 bodies, 2.27 M vertices) advanced together from rest,
each sub-scene with its own convergence, CCD bound and line search; the
line adds the same library run one scene at a time on a sample of evenly
spaced scenes over the same steps, scaled by body count, and the speedup.

    python bench.py [--steps K] [--warmup W] [--pre N]
    python bench.py --workload batched --steps 40 [--loop-scenes 16]
    python bench.py --workload adjoint --steps 100 [--checkpoint-every 10]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import scenegen as sg  # noqa: E402

FP64_PEAK_TFLOPS = 78.6   # MI355X FP64 vector, dense
HBM_PEAK_GBS = 8000.0     # MI355X HBM3E

# Algorithmic work per active pair of the barrier kernel, in FP64 operations
# (each +, -, *, /, sqrt, log counted once): case classification and
# distance ~60, barrier scalars ~25, case derivatives ~120, gradient 12, the
# 78-entry local Hessian ~1,326, the edge-edge mollifier terms ~800, the
# 9x9 translation reduction 1,224, a textbook dense symmetric eigensolve with
# vectors (9 n^3 = 6,561 for n = 9), the PSD reconstruction 810 and the map
# back to 12x12 2,106: 12,300 (point-triangle) to 13,200 (edge-edge).
BARRIER_FLOP_PER_PAIR = 12700.0
# Algorithmic bytes per CCD pair: pair ids, the 4 vertex ids and the 4
# vertices' positions and displacements.
ACCD_BYTES_PER_PAIR = 8 + 16 + 4 * 48


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--pre", type=int, default=60, help="untimed steps before warmup (spheres land)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device copy of this size (for counter calibration) before timing")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--workload", choices=("box", "batched", "adjoint"), default="box",
                    help="box: the 1000-icosphere box drop (default); batched: 256 independent drop scenes in one "
                         "launch sequence, against a per-scene loop of the same library; adjoint: gradient of a "
                         "position loss after --steps steps of the 500-icosphere drop w.r.t. the initial velocities")
    ap.add_argument("--adj-rtol", type=float, default=1e-8, help="adjoint: PCG relative residual of the adjoint solves")
    ap.add_argument("--checkpoint-every", type=int, default=10)
    ap.add_argument("--loop-scenes", type=int, default=16,
                    help="batched: scenes (evenly spaced) run one at a time for the per-scene baseline")
    ap.add_argument("--start-at", type=float, default=0.0,
                    help="start the timed steps this many seconds after process start (so a profiler's "
                         "collection period can cover exactly the timed steps)")
    return ap.parse_args()


def log(args, *a):
    if not args.quiet:
        print(*a, file=sys.stderr, flush=True)


def cpu_baseline(seconds):
    """The oracle's pair work (barrier gradient + PSD Hessian + J^T H J on the
    candidates, additive CCD on the swept candidates) on the resting bottom
    layer of the same scene, repeated for about `seconds`."""
    import oracle
    S, P = sg.icosphere_resting_layer(dhat=1e-3)
    x = oracle.vertex_map(S, S["q0"])
    q1 = sg.random_state(S, 9, rot_angle=0.05, shift=0.0)
    q1[1:, 1] -= 4e-3
    x1 = oracle.vertex_map(S, q1)
    pt, ee = oracle.candidates(S, x, None, P["dhat"])
    keys = oracle.off_keys(S, pt, ee)
    spt, see = oracle.candidates(S, x, x1, P["dhat"])
    pairs = 0
    reps = 0
    t0 = time.perf_counter()
    while True:
        r = oracle.barrier(S, x, pt, ee, P, keys, project=True)
        oracle.ccd(S, x, x1 - x, spt, see, P)
        pairs += r["n_active"] + len(spt) + len(see)
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return dict(value=pairs / el, unit="pair evals/s", cores=1, kind="oracle",
                sample=f"bottom layer of the icosphere box resting within dhat of the floor: "
                       f"{r['n_active']} active barrier pairs + {len(spt) + len(see)} CCD pairs, "
                       f"repeated {reps}x in {el:.1f} s, single thread")


def roofline(ks):
    """Roofline of the kernel with the largest live HIP-event time."""
    def per_launch(k):
        d = ks[k]
        n = max(d["launches"], 1)
        return d["ms"] / n, d["units"] / n

    dom = max(("pcg_round", "barrier_local", "accd"), key=lambda k: ks[k]["ms"])
    avg_ms, units = per_launch(dom)
    if dom == "pcg_round":
        roof = {"kernel": "pcg_round (one hipGraph replay of 16 or 64 PCG iterations, one k_cg_iter each, "
                          "+ k_cg_advance)", "bound": "hbm",
                "achieved": units / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "bytes_per_launch": units, "launches": ks[dom]["launches"]}
    elif dom == "barrier_local":
        roof = {"kernel": "k_barrier_local", "bound": "alu",
                "achieved": BARRIER_FLOP_PER_PAIR * units / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0,
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "pairs_per_launch": units}
    else:
        roof = {"kernel": "k_accd", "bound": "hbm",
                "achieved": ACCD_BYTES_PER_PAIR * units / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "pairs_per_launch": units}
    roof.update(frac=roof["achieved"] / roof["peak"], traffic=None, avg_launch_ms=avg_ms)
    bl_ms, bl_u = per_launch("barrier_local")
    ac_ms, ac_u = per_launch("accd")
    pair_kernels = {
        "barrier_local": {"avg_launch_ms": bl_ms, "pairs_per_launch": bl_u,
                          "tflops": BARRIER_FLOP_PER_PAIR * bl_u / (bl_ms * 1e-3) / 1e12 if bl_ms > 0 else 0.0,
                          "pairs_per_s": bl_u / (bl_ms * 1e-3) if bl_ms > 0 else 0.0},
        "accd": {"avg_launch_ms": ac_ms, "pairs_per_launch": ac_u,
                 "gbs": ACCD_BYTES_PER_PAIR * ac_u / (ac_ms * 1e-3) / 1e9 if ac_ms > 0 else 0.0,
                 "pairs_per_s": ac_u / (ac_ms * 1e-3) if ac_ms > 0 else 0.0}}
    return roof, pair_kernels


# HBM bytes per PCG graph replay measured on the default box-drop timed
# steps with rocprofv3 FETCH_SIZE and WRITE_SIZE (k_cg_iter + k_cg_advance,
# each counter scaled by what it reads for a 512 MiB device copy); valid for
# the k_cg_iter the measurement was taken on
PCG_ROUND_TRAFFIC = 330.3e6

KERNELS = ("pcg_round", "barrier_local", "accd", "assemble_chunks", "pair_tiles_write", "energy_only",
           "friction_local")


def timed_steps(args, ctx, sc, P, q, qd, steps):
    """steps time steps between two synchronisations, kernel timing on."""
    import torch
    ctx.profile(True, reset=True)
    torch.cuda.synchronize()
    tot = dict(newton=0, scene_newton=0, active=0, ccd=0, pcg=0, friction=0)
    t0 = time.perf_counter()
    for _ in range(steps):
        st = ctx.time_step(sc, P, q, qd)
        tot["newton"] += st["newton_iters"]
        tot["scene_newton"] += st["scene_newton_iters"]
        tot["active"] += st["n_active_pt"] + st["n_active_ee"]
        tot["ccd"] += st["n_pt_swept"] + st["n_ee_swept"]
        tot["pcg"] += st["pcg_iters"]
        tot["friction"] += st["n_friction"] * st["newton_iters"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ks = {k: ctx.profile_query(k) for k in KERNELS}
    ctx.profile(False)
    return wall, tot, ks


def wait_start(args):
    if args.start_at > 0:
        import psutil
        wait = args.start_at - (time.time() - psutil.Process().create_time())
        if wait < 0:
            log(args, f"--start-at {args.start_at}: already {-wait:.1f} s late")
        time.sleep(max(wait, 0.0))


def calib_copy(args):
    import torch
    if args.calib_copy_mib:
        # one plain device copy of known size (read + write), untimed, so
        # that HBM counters can be scaled against it
        n = args.calib_copy_mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b


def line_common(args, wall, tot, ks, steps):
    roof, pair_kernels = roofline(ks)
    pairs = tot["active"] + tot["ccd"]
    return {
        "metric": "contact-pair evals/s (barrier grad+PSD Hess+CCD, FP64); Newton iters/s",
        "value": pairs / wall,
        "unit": "pair evals/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded scene generator)",
        "newton_iters_per_s": tot["scene_newton"] / wall,
        "newton_iters": tot["scene_newton"],
        "pair_evals": {"barrier_active": tot["active"], "ccd": tot["ccd"], "friction": tot["friction"]},
        "pcg_iters": tot["pcg"],
        "kernel_ms": {k: v["ms"] for k, v in ks.items()},
        "roofline": roof,
        "pair_kernels": pair_kernels,
    }


def run_box(args):
    import torch

    import paper_2201_10022_amd as abd

    S, P = sg.icosphere_box()
    P = dict(P, max_pcg=2000)
    ctx, sc = abd.setup(S, 0)
    q = torch.as_tensor(S["q0"], device="cuda:0")
    qd = torch.as_tensor(S["qd0"], device="cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.pre):
        st = ctx.time_step(sc, P, q, qd)
        if i % 10 == 0:
            log(args, f"pre {i}: newton {st['newton_iters']} active {st['n_active_pt'] + st['n_active_ee']} "
                      f"swept {st['n_pt_swept'] + st['n_ee_swept']} pcg {st['pcg_iters']} "
                      f"{time.perf_counter() - t0:.1f}s")
    for i in range(args.warmup):
        ctx.time_step(sc, P, q, qd)
    torch.cuda.synchronize()
    wait_start(args)
    calib_copy(args)
    wall, tot, ks = timed_steps(args, ctx, sc, P, q, qd, args.steps)
    line = line_common(args, wall, tot, ks, args.steps)
    if (args.pre, args.warmup, args.steps) == (60, 2, 5) and line["roofline"]["kernel"].startswith("pcg_round"):
        # HBM bytes per replay over these timed steps (rocprofv3 FETCH_SIZE and
        # WRITE_SIZE of k_cg_iter + k_cg_advance, scaled by a 512 MiB copy)
        line["roofline"]["traffic"] = PCG_ROUND_TRAFFIC
    line["config"] = {"workload": "icosphere box drop: 1000 icospheres (subdivision 2) + fixed 12-quad box, "
                                  f"dt 1e-2, dhat 1e-3, lagged friction mu {P['mu']}",
                      "bodies": int(len(S["q0"])), "verts": int(len(S["xbar"])), "tris": int(len(S["tris"])),
                      "edges": int(len(S["edges"])), "pre_steps": args.pre}
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(line), flush=True)


def run_batched(args):
    """256 independent scenes advanced together from their first step
    (warm-up steps, then the timed steps, which include the landings),
    against the same library run on one scene at a time for a sample of
    evenly spaced scenes (same steps), scaled to all scenes."""
    import torch

    import paper_2201_10022_amd as abd

    S, P = sg.batched_drops()
    n_sc = len(S["scene_body_off"]) - 1
    steps = args.steps
    ctx, sc = abd.setup(S, 0)
    q = torch.as_tensor(S["q0"], device="cuda:0")
    qd = torch.as_tensor(S["qd0"], device="cuda:0")
    for i in range(args.warmup):
        ctx.time_step(sc, P, q, qd)
    torch.cuda.synchronize()
    wait_start(args)
    wall, tot, ks = timed_steps(args, ctx, sc, P, q, qd, steps)
    log(args, f"batched: {steps} steps in {wall:.2f} s, scene Newton iterations {tot['scene_newton']}")
    ctx.close()
    # per-scene loop on a sample of scenes
    pick = np.linspace(0, n_sc - 1, max(1, min(args.loop_scenes, n_sc))).round().astype(int)
    loop_wall, loop_newton, loop_bodies = 0.0, 0, 0
    for k in pick:
        Sk = sg.sub_scene(S, int(k))
        ck, sk = abd.setup(Sk, 0)
        qk = torch.as_tensor(Sk["q0"], device="cuda:0")
        qdk = torch.as_tensor(Sk["qd0"], device="cuda:0")
        for i in range(args.warmup):
            ck.time_step(sk, P, qk, qdk)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            st = ck.time_step(sk, P, qk, qdk)
            loop_newton += st["newton_iters"]
        torch.cuda.synchronize()
        loop_wall += time.perf_counter() - t0
        loop_bodies += len(Sk["q0"])
        ck.close()
    scale = len(S["q0"]) / loop_bodies  # by body count of the sample
    line = line_common(args, wall, tot, ks, steps)
    line["config"] = {"workload": "batched drops: 256 scenes of 2..200 cubes/icospheres over a fixed ground quad, "
                                  "dt 1e-2, dhat 1e-3, frictionless; timed steps follow the warm-up from rest",
                      "scenes": n_sc, "bodies": int(len(S["q0"])), "verts": int(len(S["xbar"])),
                      "tris": int(len(S["tris"])), "edges": int(len(S["edges"]))}
    line["per_scene_loop"] = {
        "sampled_scenes": [int(k) for k in pick], "sample_bodies": int(loop_bodies),
        "sample_wall_s": loop_wall, "sample_newton_iters": int(loop_newton),
        "scaled_wall_s": loop_wall * scale, "scale": "total bodies / sampled bodies",
        "speedup": loop_wall * scale / wall}
    print(json.dumps(line), flush=True)


def run_adjoint(args):
    """Forward rollout of the 500-icosphere drop (friction 0.5) for --steps
    steps keeping checkpoints, loss |p_1(T) - target|^2, and its gradient
    with respect to every body's initial velocity by the checkpointed
    adjoint (each segment re-run once from its checkpoint)."""
    import torch

    import paper_2201_10022_amd as abd

    S, P, target = sg.adjoint_drop()
    n = args.steps
    ctx, sc = abd.setup(S, 0)
    q0 = torch.as_tensor(S["q0"], device="cuda:0")
    qd0 = torch.as_tensor(S["qd0"], device="cuda:0")
    q, qd = q0.clone(), qd0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # forward, keeping a checkpoint every --checkpoint-every steps
    ck, newton = ctx.rollout_forward(sc, P, q, qd, n, args.checkpoint_every)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    b1 = int(np.flatnonzero(S["body_fixed"] == 0)[0])
    tq = torch.as_tensor(target, device="cuda:0")
    loss = float(((q[b1, :3] - tq) ** 2).sum())
    gT = torch.zeros_like(q)
    gT[b1, :3] = 2.0 * (q[b1, :3] - tq)
    t0 = time.perf_counter()
    gq, gqd = ctx.rollout_backward(sc, P, q0, qd0, n, args.checkpoint_every, gT, torch.zeros_like(q), args.adj_rtol,
                                   checkpoints=ck)
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    line = {"metric": "adjoint rollout: time steps differentiated per second (forward re-runs included)",
            "value": n / t_bwd, "unit": "steps/s", "n_gpus": 1, "steps": n, "warmup": 0,
            "ms_per_step": 1e3 * t_bwd / max(n, 1), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded scene generator)",
            "config": {"workload": "adjoint drop: 500 icospheres (5 layers) in the fixed box, lagged friction "
                                   f"mu {P['mu']}, loss |p_1(T) - target|^2, gradient w.r.t. all initial "
                                   "velocities", "bodies": int(len(S["q0"])),
                       "checkpoint_every": args.checkpoint_every, "adjoint_pcg_rtol": args.adj_rtol},
            "forward_s": t_fwd, "backward_s": t_bwd, "backward_over_forward": t_bwd / t_fwd,
            "forward_newton_iters": newton, "loss": loss,
            "grad_qdot0_norm": float(gqd.norm()), "grad_q0_norm": float(gq.norm())}
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: multi-GPU execution is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "batched":
        run_batched(args)
    elif args.workload == "adjoint":
        run_adjoint(args)
    else:
        run_box(args)


if __name__ == "__main__":
    main()

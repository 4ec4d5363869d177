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

    python bench.py [--steps K] [--warmup W] [--pre N]
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

# Algorithmic work per active pair of the barrier kernel (counted stage by
# stage in the design doc): case classification and distance, barrier scalars,
# case derivatives, the 78-entry local Hessian, the 9x9 translation
# reduction, a textbook dense symmetric eigensolve with vectors (9 n^3,
# n = 9), the PSD reconstruction and the map back to 12x12.
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


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)
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
    if args.start_at > 0:
        import psutil
        wait = args.start_at - (time.time() - psutil.Process().create_time())
        if wait < 0:
            log(args, f"--start-at {args.start_at}: already {-wait:.1f} s late")
        time.sleep(max(wait, 0.0))
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
    ctx.profile(True, reset=True)
    torch.cuda.synchronize()
    tot = dict(newton=0, active=0, ccd=0, pcg=0, friction=0)
    t0 = time.perf_counter()
    for i in range(args.steps):
        st = ctx.time_step(sc, P, q, qd)
        tot["newton"] += st["newton_iters"]
        tot["active"] += st["n_active_pt"] + st["n_active_ee"]
        tot["ccd"] += st["n_pt_swept"] + st["n_ee_swept"]
        tot["pcg"] += st["pcg_iters"]
        tot["friction"] += st["n_friction"] * st["newton_iters"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ks = {k: ctx.profile_query(k) for k in ("pcg_round", "barrier_local", "accd", "assemble_chunks",
                                             "pair_tiles_write", "energy_only", "friction_local")}
    ctx.profile(False)
    pairs = tot["active"] + tot["ccd"]

    def per_launch(k):
        d = ks[k]
        n = max(d["launches"], 1)
        return d["ms"] / n, d["units"] / n

    # dominant kernel by live HIP-event time over the timed steps
    dom = max(("pcg_round", "barrier_local", "accd"), key=lambda k: ks[k]["ms"])
    avg_ms, units = per_launch(dom)
    if dom == "pcg_round":
        roof = {"kernel": "pcg_round (one hipGraph replay: 16 x (k_pcg_spmv + k_pcg_update))", "bound": "hbm",
                "achieved": units / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "bytes_per_launch": units}
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
    line = {
        "metric": "contact-pair evals/s (barrier grad+PSD Hess+CCD, FP64); Newton iters/s",
        "value": pairs / wall,
        "unit": "pair evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded scene generator)",
        "config": {"workload": "icosphere box drop: 1000 icospheres (subdivision 2) + fixed 12-quad box, "
                               f"dt 1e-2, dhat 1e-3, lagged friction mu {P['mu']}",
                   "bodies": int(len(S["q0"])), "verts": int(len(S["xbar"])), "tris": int(len(S["tris"])),
                   "edges": int(len(S["edges"])), "pre_steps": args.pre},
        "newton_iters_per_s": tot["newton"] / wall,
        "newton_iters": tot["newton"],
        "pair_evals": {"barrier_active": tot["active"], "ccd": tot["ccd"], "friction": tot["friction"]},
        "pcg_iters": tot["pcg"],
        "kernel_ms": {k: v["ms"] for k, v in ks.items()},
        "roofline": roof,
        "pair_kernels": pair_kernels,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

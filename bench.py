"""Throughput of the affine-body contact path on one MI355X.

Default workload (the largest single-GPU configuration): 256 independent
drop scenes advanced together, scene k holding 2..200 cubes or icospheres
(26,914 bodies, 2.27 M vertices, 4.42 M triangles, 6.64 M edges, FP64)
over its own fixed ground quad.  A step is one implicit-Euler time step of
the whole batch: every Newton iteration runs the kinematic map, both
candidate sweeps, the barrier gradient and PSD-projected Hessian with
J^T H J assembly, the body terms, the PCG solve, CCD and the line search,
each sub-scene with its own convergence test, CCD bound, line search and
PCG scalars.  The timed steps follow --warmup steps from rest and include
the first layers' landings.

Printed JSON line: value = contact-pair evaluations per second (active
pairs through the barrier kernels plus pairs through CCD, summed over
every Newton iteration of every scene in the timed steps, divided by the
timed wall-clock), plus Newton iterations per second, the roofline
position of the dominant kernel (HIP events inside the library; measured
HBM traffic from the committed counter summary of the same command while
the kernel's source is unchanged), the same library run one scene at a
time on a sample of scenes, the CPU oracle's rate on a bounded sample of
the same work, and shorter runs of the other two single-scene workloads.

Other workloads:
    --workload box      the 1000-icosphere box drop (162,017 vertices,
                        lagged friction), timed after the spheres landed
    --workload chains   64 interlocked links in 8 chains (640,000
                        vertices), dt 5e-3, dhat 5e-4
    --workload wrecking a ball on an 8-link chain swung into a wall of 560
                        cubes (570 bodies), timed over the impact
    --workload adjoint  gradient of a position loss after --steps steps of
                        the 500-icosphere drop w.r.t. the initial velocities

    python bench.py [--steps K] [--warmup W] [--no-extras] [--no-cpu]
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
# vertices' positions at the start and the end of the step.
ACCD_BYTES_PER_PAIR = 8 + 16 + 4 * 48


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--pre", type=int, default=60, help="untimed steps before warmup (spheres land)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="batched: skip the short runs of the box-drop and chain workloads")
    ap.add_argument("--timed-only", action="store_true",
                    help="batched: print the line right after the timed steps (no per-scene loop, extras or CPU "
                         "baseline), so that a profiler sees nothing after them")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device copy of this size (for counter calibration) before timing")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--workload", choices=("batched", "box", "chains", "wrecking", "adjoint"), default="batched",
                    help="batched: 256 independent drop scenes in one launch sequence, against a per-scene loop "
                         "of the same library (default); box: the 1000-icosphere box drop; chains: 64 "
                         "interlocked links; wrecking: a ball on a chain swung into a wall of 560 cubes; "
                         "adjoint: gradient of a position loss after --steps steps of the "
                         "500-icosphere drop w.r.t. the initial velocities")
    ap.add_argument("--adj-rtol", type=float, default=1e-8, help="adjoint: PCG relative residual of the adjoint solves")
    ap.add_argument("--checkpoint-every", type=int, default=10)
    ap.add_argument("--loop-scenes", type=int, default=8,
                    help="batched: scenes (evenly spaced) run one at a time for the per-scene baseline")
    ap.add_argument("--tune", choices=("table", "auto", "default"), default="table",
                    help="launch shapes: the committed autotuned table for the workload (default), a fresh "
                         "autotuner run on the workload's state after the warm-up (untimed), or the library's "
                         "defaults")
    ap.add_argument("--tune-steps", type=int, default=10, help="--tune auto: time steps per trial")
    ap.add_argument("--start-at", type=float, default=0.0,
                    help="start the timed steps this many seconds after process start (so a profiler's "
                         "collection period can cover exactly the timed steps)")
    return ap.parse_args()


def log(args, *a):
    if not args.quiet:
        print(*a, file=sys.stderr, flush=True)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def batched_sample(S, P, n_pick=16):
    """n_pick evenly spaced scenes of the batch at the landing of their
    lowest layer (the CPU baseline's sample)."""
    n_sc = len(S["scene_body_off"]) - 1
    pick = np.linspace(0, n_sc - 1, min(n_pick, n_sc)).round().astype(int)
    return ([sg.landed(sg.sub_scene(S, int(k)), seed=1000 + int(k), dhat=P["dhat"]) for k in pick],
            f"{len(pick)} evenly spaced scenes of the batch")


def cpu_baseline(seconds, scenes, P):
    """The oracle (OpenMP over pairs and bodies, all host threads) doing the
    same work as the GPU step on a bounded sample of it: whole Newton
    iterations (incremental potential with barrier gradient and projected
    Hessian, direct solve, swept candidates, CCD, line search) of the
    sampled scenes at the moment their lowest layer lands (bodies
    U[0.2,0.8] dhat above the ground, moving down at 1 m/s), repeated until
    about `seconds` have passed.  value = (active barrier pairs + CCD
    pairs) / wall time of those iterations, the GPU value's definition;
    pair_work_only divides the same pairs by the time of the barrier and
    CCD calls alone."""
    import oracle
    scenes, what = scenes
    work = []
    for Sk in scenes:
        Bk = oracle.Body(Sk)
        qt = oracle.q_tilde(Sk, Sk["q0"], Sk["qd0"], P)
        work.append((Sk, Bk, qt, oracle.step_friction(Sk, Sk["q0"], P)))
    pairs, iters, reps, el = 0, 0, 0, 0.0
    t0 = time.perf_counter()
    while el < seconds:
        for Sk, Bk, qt, F in work:
            _, conv, info = oracle.newton_iteration(Sk, Bk, Sk["q0"], qt, P, F)
            pairs += info["n_active"] + info.get("n_pt_swept", 0) + info.get("n_ee_swept", 0)
            iters += 1
        reps += 1
        el = time.perf_counter() - t0
    # the pair work alone (barrier + CCD calls on the same pairs), one pass
    pw_pairs, pw_t = 0, 0.0
    for Sk, Bk, qt, F in work:
        q = Sk["q0"]
        x = oracle.vertex_map(Sk, q)
        pt, ee = oracle.candidates(Sk, x, None, P["dhat"])
        keys = oracle.off_keys(Sk, pt, ee)
        gh = oracle.grad_hess(Sk, Bk, q, qt, P, x=x, pt=pt, ee=ee, F=F)
        p = oracle.solve(Sk, gh["diag"], gh["off"], gh["keys"], -gh["grad"])
        x1 = oracle.vertex_map(Sk, q + p)
        spt, see = oracle.candidates(Sk, x, x1, P["dhat"])
        t1 = time.perf_counter()
        r = oracle.barrier(Sk, x, pt, ee, P, keys, project=True)
        oracle.ccd(Sk, x, x1 - x, spt, see, P)
        pw_t += time.perf_counter() - t1
        pw_pairs += r["n_active"] + len(spt) + len(see)
    return dict(value=pairs / el, unit="pair evals/s", cores=oracle.threads(), kind="oracle",
                cpu_model=_cpu_model(), newton_iters_per_s=iters / el,
                pair_work_only={"value": pw_pairs / pw_t if pw_t > 0 else 0.0,
                                "denominator": "time of the oracle's barrier and CCD calls only"},
                sample=f"{what} ({sum(len(w[0]['q0']) for w in work)} "
                       f"bodies) at the landing of their lowest layer: one Newton iteration each, repeated "
                       f"{reps}x ({iters} iterations, {pairs} pair evaluations) in {el:.1f} s on "
                       f"{oracle.threads()} OpenMP threads")


def roofline(ks):
    """Roofline of the kernel with the largest live HIP-event time."""
    def per_launch(k):
        d = ks[k]
        n = max(d["launches"], 1)
        return d["ms"] / n, d["units"] / n

    dom = max(("pcg_round", "barrier_local", "accd"), key=lambda k: ks[k]["ms"])
    avg_ms, units = per_launch(dom)
    if dom == "pcg_round":
        roof = {"kernel": "pcg_round (one hipGraph replay of pcg_short or pcg_long PCG iterations of the launch "
                          "table, one k_cg_iter each, + k_cg_compact for a batch + k_cg_advance)", "bound": "hbm",
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


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 counter summaries (profiles/*.md, a line
    `bench-traffic: kernel=K workload=W bytes_per_launch=B sources=F1,F2
    sha256=H`), or None when there is none or when the kernel's sources
    have changed since the counters were taken (H is the SHA-256 of the
    listed source files' contents, concatenated in order)."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as f:
            for line in f:
                if not line.startswith("bench-traffic:"):
                    continue
                kv = dict(t.split("=", 1) for t in line.split()[1:] if "=" in t)
                if kv.get("kernel") != kernel or kv.get("workload") != workload:
                    continue
                h = hashlib.sha256()
                for src in kv.get("sources", "").split(","):
                    with open(os.path.join(ROOT, src), "rb") as g:
                        h.update(g.read())
                if h.hexdigest() != kv.get("sha256"):
                    return None, f"{os.path.basename(path)}: sources changed since the counters were taken"
                return float(kv["bytes_per_launch"]), os.path.basename(path)
    return None, "no counter summary for this kernel and workload"


KERNELS = ("pcg_round", "barrier_local", "accd", "assemble_chunks", "pair_tiles_write", "energy_only",
           "friction_local")
# host-side work inside the timed steps: workspace growth (synchronise, free,
# allocate, clear) and captures of the PCG graphs
HOST_EVENTS = ("ws_grow", "pcg_capture")


def timed_steps(args, ctx, sc, P, q, qd, steps):
    """steps time steps between two synchronisations, kernel timing on."""
    import torch
    ctx.profile(True, reset=True)
    torch.cuda.synchronize()
    tot = dict(newton=0, scene_newton=0, active=0, ccd=0, pcg=0, friction=0,
               host_ms=dict(candidates=0.0, barrier=0.0, solve=0.0, ccd_line_search=0.0, total=0.0))
    t0 = time.perf_counter()
    for _ in range(steps):
        st = ctx.time_step(sc, P, q, qd)
        for k, f in (("candidates", "t_candidates_ms"), ("barrier", "t_barrier_ms"), ("solve", "t_solve_ms"),
                     ("ccd_line_search", "t_ccd_ms"), ("total", "t_total_ms")):
            tot["host_ms"][k] += st[f]
        tot["newton"] += st["newton_iters"]
        tot["scene_newton"] += st["scene_newton_iters"]
        tot["active"] += st["n_active_pt"] + st["n_active_ee"]
        tot["ccd"] += st["n_pt_swept"] + st["n_ee_swept"]
        tot["pcg"] += st["pcg_iters"]
        tot["friction"] += st["n_friction"] * st["newton_iters"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ks = {k: ctx.profile_query(k) for k in KERNELS}
    tot["host_events"] = {k: ctx.profile_query(k) for k in HOST_EVENTS}
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
        "phase_wall_ms": {k: v / steps for k, v in tot["host_ms"].items()},
        "host_events": {k: {"count": v["launches"], "ms": v["ms"]} for k, v in tot["host_events"].items()},
        "kernel_ms": {k: v["ms"] for k, v in ks.items()},
        "roofline": roof,
        "pair_kernels": pair_kernels,
    }


TUNE_TABLE = os.path.join(ROOT, "paper_2201_10022_amd", "tune_mi355x.json")


def apply_tune(args, ctx, sc, P, q, qd, workload):
    """Sets the context's launch-shape table; returns (table, source)."""
    if args.tune == "default":
        return ctx.tune_get(), "library defaults"
    if args.tune == "auto":
        table, ms = ctx.autotune(sc, P, q, qd, n_steps=args.tune_steps, reps=2)
        return table, f"autotuned in this run ({ms:.2f} ms per step over {args.tune_steps} steps from here)"
    entry = None
    if os.path.exists(TUNE_TABLE):
        with open(TUNE_TABLE) as f:
            entry = json.load(f).get(workload)
    if entry is None:
        return ctx.tune_get(), "library defaults (no committed table for this workload)"
    ctx.tune_set(entry["table"])
    return ctx.tune_get(), "committed autotuned table (paper_2201_10022_amd/tune_mi355x.json)"


def attach_traffic(line, workload):
    roof = line["roofline"]
    kname = "pcg_round" if roof["kernel"].startswith("pcg_round") else roof["kernel"]
    t, src = measured_traffic(kname, workload)
    roof["traffic"] = t
    roof["traffic_source"] = src


def box_line(args, pre, warmup, steps, quiet=False):
    """The 1000-icosphere box drop: `pre` untimed steps (the spheres land),
    `warmup` more, then `steps` timed steps."""
    import torch

    import paper_2201_10022_amd as abd

    S, P = sg.icosphere_box()
    P = dict(P, max_pcg=2000)
    ctx, sc = abd.setup(S, 0)
    q = torch.as_tensor(S["q0"], device="cuda:0")
    qd = torch.as_tensor(S["qd0"], device="cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(pre):
        st = ctx.time_step(sc, P, q, qd)
        if i % 10 == 0 and not quiet:
            log(args, f"box pre {i}: newton {st['newton_iters']} active {st['n_active_pt'] + st['n_active_ee']} "
                      f"swept {st['n_pt_swept'] + st['n_ee_swept']} pcg {st['pcg_iters']} "
                      f"{time.perf_counter() - t0:.1f}s")
    for i in range(warmup):
        ctx.time_step(sc, P, q, qd)
    tune = apply_tune(args, ctx, sc, P, q, qd, "box")
    torch.cuda.synchronize()
    wall, tot, ks = timed_steps(args, ctx, sc, P, q, qd, steps)
    ctx.close()
    line = line_common(args, wall, tot, ks, steps)
    line["warmup"] = warmup
    line["tune"] = {"table": tune[0], "source": tune[1]}
    line["config"] = {"workload": "icosphere box drop: 1000 icospheres (subdivision 2) + fixed 12-quad box, "
                                  f"dt 1e-2, dhat 1e-3, lagged friction mu {P['mu']}",
                      "bodies": int(len(S["q0"])), "verts": int(len(S["xbar"])), "tris": int(len(S["tris"])),
                      "edges": int(len(S["edges"])), "pre_steps": pre}
    line["steps_per_s"] = steps / wall
    attach_traffic(line, "box")
    return line


def chains_line(args, warmup, steps):
    """The chain workload from its initial state: `warmup` untimed steps,
    then `steps` timed steps."""
    import torch

    import paper_2201_10022_amd as abd

    S, P = sg.torus_chains()
    ctx, sc = abd.setup(S, 0)
    q = torch.as_tensor(S["q0"], device="cuda:0")
    qd = torch.as_tensor(S["qd0"], device="cuda:0")
    for i in range(warmup):
        ctx.time_step(sc, P, q, qd)
    tune = apply_tune(args, ctx, sc, P, q, qd, "chains")
    torch.cuda.synchronize()
    wall, tot, ks = timed_steps(args, ctx, sc, P, q, qd, steps)
    ctx.close()
    line = line_common(args, wall, tot, ks, steps)
    line["warmup"] = warmup
    line["tune"] = {"table": tune[0], "source": tune[1]}
    line["config"] = {"workload": "interlocked chains: 8 chains x 8 links (major 0.3, minor 0.1, 200 x 50 "
                                  "grid, stadium links), end links fixed, dt 5e-3, dhat 5e-4, frictionless",
                      "bodies": int(len(S["q0"])), "verts": int(len(S["xbar"])), "tris": int(len(S["tris"])),
                      "edges": int(len(S["edges"]))}
    line["steps_per_s"] = steps / wall
    attach_traffic(line, "chains")
    return line


def wrecking_line(args, pre, warmup, steps):
    """The wrecking-ball-shaped workload: `pre` untimed steps (the ball
    swings down), `warmup` more, then `steps` timed steps (the impact)."""
    import torch

    import paper_2201_10022_amd as abd

    S, P = sg.wrecking_ball()
    ctx, sc = abd.setup(S, 0)
    q = torch.as_tensor(S["q0"], device="cuda:0")
    qd = torch.as_tensor(S["qd0"], device="cuda:0")
    for i in range(pre + warmup):
        ctx.time_step(sc, P, q, qd)
    tune = apply_tune(args, ctx, sc, P, q, qd, "wrecking")
    torch.cuda.synchronize()
    wall, tot, ks = timed_steps(args, ctx, sc, P, q, qd, steps)
    ctx.close()
    line = line_common(args, wall, tot, ks, steps)
    line["warmup"] = warmup
    line["tune"] = {"table": tune[0], "source": tune[1]}
    line["config"] = {"workload": "wrecking ball: wall of 560 cubes on a ground quad, 65 kg ball with an eyelet on "
                                  "an 8-link chain from a fixed pivot, swung 60 degrees, dt 1e-2, dhat 1e-3, "
                                  "frictionless", "bodies": int(len(S["q0"])), "verts": int(len(S["xbar"])),
                      "tris": int(len(S["tris"])), "edges": int(len(S["edges"])), "pre_steps": pre}
    line["steps_per_s"] = steps / wall
    attach_traffic(line, "wrecking")
    return line


def run_wrecking(args):
    wait_start(args)
    line = wrecking_line(args, args.pre if args.pre != 60 else 40, args.warmup, args.steps)
    print(json.dumps(line), flush=True)


def culling_ops(args, reps=10):
    """The candidate search (body boxes, i-AABB lists, tiled primitive-pair
    box tests, both passes) with the single i-AABB and with the three-level
    tree per i-AABB (sec. 4.2, Fig. iBVH), on the interlocked links in
    contact swept over one step of their initial velocities (entangled: the
    links' i-AABBs hold whole arcs of both tori) and on the box drop's
    landing state: host wall time per call (the call synchronises to read
    its counts), best of `reps`, and the primitive-pair box tests each
    runs.  Both give the same pairs in the same order."""
    import torch

    import paper_2201_10022_amd as abd

    out = {}
    for name, make in (("chains", lambda: sg.torus_chains()), ("box", lambda: sg.icosphere_box())):
        S, P = make()
        if name == "chains":
            q = sg.torus_chains_contact(S, 8)
        else:
            S = sg.landed(S, seed=7, dhat=P["dhat"])
            q = S["q0"]
        ctx, sc = abd.setup(S, 0)
        qg = torch.as_tensor(q, device="cuda:0")
        q1 = torch.as_tensor(q + P["dt"] * S["qd0"], device="cuda:0")
        x0, x1 = ctx.vertex_map(sc, qg), ctx.vertex_map(sc, q1)
        res = {}
        for levels in (1, 3):
            ctx.tune_set(dict(cull_levels=levels))
            ctx.candidates(sc, x0, x1, P["dhat"])
            ctx.profile(2, True)
            pt, ee = ctx.candidates(sc, x0, x1, P["dhat"])
            tests = ctx.profile_query("box_tests")["units"]
            ctx.profile(False, True)
            best = float("inf")
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx.candidates(sc, x0, x1, P["dhat"])
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t0)
            res[f"levels_{levels}"] = {"ms_per_call": 1e3 * best, "box_tests": int(tests),
                                       "pairs": int(len(pt) + len(ee))}
        ctx.close()
        res["tests_tree_over_single"] = res["levels_3"]["box_tests"] / max(res["levels_1"]["box_tests"], 1)
        res["time_tree_over_single"] = res["levels_3"]["ms_per_call"] / res["levels_1"]["ms_per_call"]
        out[name] = res
    return out


def rigidity_ops(args, reps=50):
    """Energy operations of the three rigidity potentials (energy, gradient
    and PSD-projected 9x9 Hessian per body; sec. 3.2 compares V_perp with
    ARAP and neo-Hookean) on the batched workload's 26,914 bodies, each A a
    seeded random rotation times (I + 0.05 N(0,1)): mean kernel time per
    call from torch events on the library's stream, and the time of each
    alternative over V_perp's."""
    import torch

    import paper_2201_10022_amd as abd

    S, P = sg.batched_drops()
    ctx, sc = abd.setup(S, 0)
    rng = np.random.default_rng(11)
    q = S["q0"].copy()
    for b in np.flatnonzero(S["body_fixed"] == 0):
        Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        q[b, 3:] = (Q * np.sign(np.linalg.det(Q)) @ (np.eye(3) + 0.05 * rng.normal(size=(3, 3)))).reshape(9)
    import ctypes
    qg = torch.as_tensor(q, device="cuda:0")
    nbt = len(S["q0"])
    e = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    g = torch.zeros((nbt, 12), dtype=torch.float64, device="cuda:0")
    D = torch.zeros((nbt, 144), dtype=torch.float64, device="cuda:0")
    out = {}
    for kind, name in ((0, "orthogonality"), (1, "arap"), (2, "neo_hookean")):
        prm = abd.make_params(dict(P, rigidity=kind))

        def call():
            # (accumulates into the same buffers: only the library's kernels run)
            ctx._check(ctx.L.abd_orthogonality(ctx.h, ctypes.byref(sc.c), ctypes.byref(prm), abd._ptr(qg),
                                               P["dt"] ** 2, abd._ptr(e), abd._ptr(g), abd._ptr(D), 1,
                                               abd._stream()))
        for _ in range(3):
            call()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            call()
        b.record()
        torch.cuda.synchronize()
        out[name] = {"ms_per_call": a.elapsed_time(b) / reps}
    ctx.close()
    nb = int((S["body_fixed"] == 0).sum())
    base = out["orthogonality"]["ms_per_call"]
    for name, v in out.items():
        v["ns_per_body"] = 1e6 * v["ms_per_call"] / nb
        v["time_over_orthogonality"] = v["ms_per_call"] / base
    out["bodies"] = nb
    out["op"] = ("energy + gradient + PSD-projected Hessian per body (one abd_orthogonality call: the body-terms "
                 "kernel and the energy sum)")
    return out


def run_box(args):
    wait_start(args)
    calib_copy(args)
    line = box_line(args, args.pre, args.warmup, args.steps)
    if not args.no_cpu:
        S, P = sg.icosphere_box(n_layers=2)
        sample = ([sg.landed(S, seed=1000, dhat=P["dhat"])], "the box drop's lowest 2 of 10 layers (200 spheres)")
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds, sample, P)
    print(json.dumps(line), flush=True)


def run_chains(args):
    wait_start(args)
    calib_copy(args)
    line = chains_line(args, args.warmup, args.steps)
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
    tune = apply_tune(args, ctx, sc, P, q, qd, "batched")
    torch.cuda.synchronize()
    wait_start(args)
    calib_copy(args)
    wall, tot, ks = timed_steps(args, ctx, sc, P, q, qd, steps)
    log(args, f"batched: {steps} steps in {wall:.2f} s, scene Newton iterations {tot['scene_newton']}")
    ctx.close()
    line = line_common(args, wall, tot, ks, steps)
    line["config"] = {"workload": "batched drops: 256 scenes of 2..200 cubes/icospheres over a fixed ground quad, "
                                  "dt 1e-2, dhat 1e-3, frictionless; timed steps follow the warm-up from rest",
                      "scenes": n_sc, "bodies": int(len(S["q0"])), "verts": int(len(S["xbar"])),
                      "tris": int(len(S["tris"])), "edges": int(len(S["edges"]))}
    line["steps_per_s"] = steps / wall
    line["tune"] = {"table": tune[0], "source": tune[1]}
    attach_traffic(line, "batched")
    if args.timed_only:
        print(json.dumps(line), flush=True)
        return
    # per-scene loop on a sample of scenes
    pick = np.linspace(0, n_sc - 1, max(1, min(args.loop_scenes, n_sc))).round().astype(int)
    loop_wall, loop_newton, loop_bodies = 0.0, 0, 0
    for k in pick:
        Sk = sg.sub_scene(S, int(k))
        ck, sk = abd.setup(Sk, 0)
        ck.tune_set(tune[0])
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
    line["per_scene_loop"] = {
        "sampled_scenes": [int(k) for k in pick], "sample_bodies": int(loop_bodies),
        "sample_wall_s": loop_wall, "sample_newton_iters": int(loop_newton),
        "scaled_wall_s": loop_wall * scale, "scale": "total bodies / sampled bodies",
        "speedup": loop_wall * scale / wall}
    if not args.no_extras:
        log(args, "extra: box drop")
        bl = box_line(args, 60, 2, 5, quiet=True)
        log(args, "extra: chains")
        cl = chains_line(args, 2, 5)
        log(args, "extra: wrecking ball")
        wl = wrecking_line(args, 40, 2, 10)
        keep = ("value", "unit", "ms_per_step", "steps_per_s", "newton_iters_per_s", "newton_iters", "steps",
                "warmup", "pair_evals", "pcg_iters", "roofline", "pair_kernels", "config")
        line["other_configs"] = {"box": {k: bl[k] for k in keep}, "chains": {k: cl[k] for k in keep},
                                 "wrecking": {k: wl[k] for k in keep}}
        log(args, "extra: rigidity potentials")
        line["rigidity_ops"] = rigidity_ops(args)
        log(args, "extra: i-AABB culling levels")
        line["culling_ops"] = culling_ops(args)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds, batched_sample(S, P), P)
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
    elif args.workload == "chains":
        run_chains(args)
    elif args.workload == "wrecking":
        run_wrecking(args)
    else:
        run_box(args)


if __name__ == "__main__":
    main()

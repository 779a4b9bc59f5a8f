"""Benchmark of the MDF-FDLBM FP64 time step on one MI355X.

Workload: lid-driven square cavity, Re = 1000, 1024 x 1024 nodes (walls
included), lid speed 0.1, fluid at rest initially, FP64 throughout.  A "step"
is one full time step of the method (Steps (1)-(4) of Sec. 2.2 with walls).

Prints one JSON line with MLUPS (= nodes x steps / s / 1e6), the roofline of
the fused step kernel (algorithmic 160 B per node and step: one read and one
write of the ten FP64 distribution planes) and the CPU oracle timed on a
bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E peak
BYTES_PER_NODE = 160.0         # 10 FP64 planes read + 10 written per node and step
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_2306_08216_amd", "csrc")
TUNING = os.path.join(ROOT, "paper_2306_08216_amd", "tuning_mi355x.json")
METRIC = "MLUPS (FP64) + % HBM roofline; learned-closure speedup at equal L2 error"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sha():
    """Digest of the step's sources (kernels, device header, launch plan); a
    counter summary taken on other sources no longer describes these kernels."""
    h = hashlib.sha256()
    for f in ("mdf_fused.hip", "mdf_fused2.hip", "mdf_device.hpp", "mdf_internal.hpp", "mdf_api.hip"):
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()[:16]


def choice_text(choice):
    """(variant, tile_w, prefetch, x scale, y scale) as the counter summaries write it."""
    v, tw, pf, sx, sy = choice
    return f"{int(v)} {int(tw)} {int(pf)} {float(sx):g} {float(sy):g}"


def measured_traffic(workload, n, choice):
    """HBM bytes per launch from the committed rocprofv3 counter summary of this
    workload, if it was taken on the current sources with the same kernel
    choice; else None."""
    path = os.path.join(PROFILES, f"fused_step_{workload}{n}_traffic.md")
    if choice is None or not os.path.exists(path):
        return None
    txt = open(path).read()
    m_sha = re.search(r"kernel_sha:\s*([0-9a-f]+)", txt)
    m_ch = re.search(r"choice:\s*([^\n]+)", txt)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not (m_sha and m_ch and m_b) or m_sha.group(1) != kernel_sha() or m_ch.group(1).strip() != choice_text(choice):
        return None
    return float(m_b.group(1))


def measured_batch_traffic(choice):
    """HBM bytes per batched step from the committed counter summary, if taken
    on the current sources with the same (variant, prefetch, rounds, tile_w)."""
    path = os.path.join(PROFILES, "fused_step_batch256_traffic.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_sha = re.search(r"kernel_sha:\s*([0-9a-f]+)", txt)
    m_ch = re.search(r"choice:\s*([^\n]+)", txt)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    want = " ".join(str(int(v)) for v in choice)
    if not (m_sha and m_ch and m_b) or m_sha.group(1) != kernel_sha() or m_ch.group(1).strip() != want:
        return None
    return float(m_b.group(1))


def cpu_baseline(prob, steps):
    """The CPU oracle (single thread, as it stands) on `steps` steps of the same workload."""
    from oracle.orc import Oracle
    o = Oracle(prob)
    o.step(1)
    t0 = time.perf_counter()
    o.step(steps)
    el = time.perf_counter() - t0
    return prob.nodes * steps / el / 1e6, el


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--n", type=int, default=1024, help="nodes per side")
    ap.add_argument("--workload", choices=["cavity", "taylor-green", "powerlaw", "batch"], default="cavity",
                    help="cavity: the benchmarked lid-driven cavity; taylor-green: periodic decaying "
                         "vortex of the same size (wall-free comparison); powerlaw: power-law cavity "
                         "(n = 0.5) on a tanh-stretched grid; batch: 256 periodic decaying-vortex instances "
                         "of sizes 64..512 advanced together (one launch per step)")
    ap.add_argument("--pl-n", type=float, default=0.5, choices=[0.5, 1.5],
                    help="power-law index of the powerlaw workload")
    ap.add_argument("--tile-w", type=int, default=0)
    ap.add_argument("--seg-h", type=int, default=0,
                    help="rows per segment; -r: the balanced plan over r rounds of workgroups (0: library default)")
    ap.add_argument("--variant", type=int, default=-1,
                    help="step kernel: 0 three-pass, 1 fused one wave per strip, 2 fused one wave per "
                         "velocity component (-1: the library's default for the workload)")
    ap.add_argument("--cpu-steps", type=int, default=40, help="oracle steps for the CPU baseline (0 = skip)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the library's autotuner (run before the warm-up, outside the timed region)")
    ap.add_argument("--tuning", default=TUNING,
                    help="tuning cache: a kernel choice stored for this workload and device is used as is; "
                         "otherwise the autotuner runs and its choice is stored")
    ap.add_argument("--retune", action="store_true", help="run the autotuner even if the cache holds a choice")
    ap.add_argument("--prefetch", type=int, default=0, help="rows prefetched by the fused kernel (2 or 3)")
    ap.add_argument("--cost-scales", default="",
                    help="x,y scalings of the wall-row costs in the balanced partition (instead of autotuning)")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="after timing, run this many plain state copies (mdf_save: 80 B read + 80 B written "
                         "per node) as the known-size reference for HBM byte counters")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "the MDF-FDLBM step runs on exactly one GPU here; multi-GPU runs are not supported",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch

    from paper_2306_08216_amd import problems as P
    from paper_2306_08216_amd.solver import Solver

    if args.workload == "batch":
        return bench_batch(args)

    if args.workload == "cavity":
        prob = P.cavity(args.n, re=1000.0, lid=0.1)
        wl = f"lid-driven cavity Re=1000, {args.n}x{args.n} nodes, lid 0.1, from rest, FP64"
    elif args.workload == "powerlaw":
        prob = P.powerlaw_cavity(args.n, pl_n=args.pl_n)
        wl = f"power-law cavity n={args.pl_n:g}, tanh-stretched {args.n}x{args.n} grid, Re_PL=100, lid 0.1, FP64"
    else:
        prob = P.taylor_green(args.n, u0=0.01, nu=0.01)
        wl = f"periodic Taylor-Green vortex, {args.n}x{args.n} nodes, u0 0.01, nu 0.01, FP64"
    dev = torch.device("cuda:0")
    s = Solver(prob, device="cuda:0")
    # warm-up first, so that a tuning run sees the flow the timed steps see (a
    # power-law collision costs less where the fluid is still at rest); the
    # autotuner restores the state it starts from
    s.step(args.warmup)
    torch.cuda.synchronize(dev)
    tuned = None
    choice = None
    if args.variant >= 0 or args.tile_w or args.seg_h or args.prefetch or args.cost_scales:
        variant = args.variant if args.variant >= 0 else (1 if prob.pl_n != 1.0 else 2)
        s.set_kernel(variant, args.tile_w, args.seg_h, args.prefetch)
        cx = cy = 1.0
        if args.cost_scales:
            cx, cy = (float(t) for t in args.cost_scales.split(","))
            s.set_partition_costs(cx, cy)
        if variant in (1, 2) and args.seg_h <= 0:
            choice = (variant, 64 if variant == 2 else (args.tile_w or 64), args.prefetch or 2, cx, cy)
    elif not args.no_autotune:
        choice, cached = s.tuned(args.tuning, steps=40, retune=args.retune)
        variant = int(choice[0])
        tuned = {"variant": variant, "tile_w": choice[1], "prefetch": choice[2], "x_wall_cost_scale": choice[3],
                 "y_wall_cost_scale": choice[4], "from_cache": cached}
    else:
        variant = 1 if prob.pl_n != 1.0 else 2
    rounds = -args.seg_h if args.seg_h < 0 else 1
    partition = (f"seg_h={args.seg_h}" if args.seg_h > 0 else
                 f"balanced segment table, {rounds} round{'s' if rounds > 1 else ''} of workgroups")
    tile_w = int(choice[1]) if choice else (args.tile_w or 64)
    kname = {0: "three-pass (k_bar_plus, k_mid, k_hat_new)",
             1: "k_fused (one wave per strip)" if tile_w == 64 else f"k_fused ({tile_w}-lane strips, one wave per 64)",
             2: "k_fused2 (one wave per velocity component)"}[variant]
    stream = s.stream

    s.step(5)   # first launches of the chosen kernel outside the timing
    torch.cuda.synchronize(dev)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    ev0.record(stream)
    s.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    diag, status = s.diagnostics()
    if status != 0:
        log(f"warning: diagnostics status {status}: {diag}")

    if args.copy_calib > 0:
        for _ in range(args.copy_calib):
            s.save()
        torch.cuda.synchronize(dev)

    nodes = prob.nodes
    sec = gpu_ms / 1e3
    mlups = nodes * args.steps / sec / 1e6
    # one step-kernel launch per step on the context's stream, plus one wall-rule
    # launch per mdf_step call (a few microseconds once per timed region)
    launch_s = sec / args.steps
    achieved = BYTES_PER_NODE * nodes / launch_s / 1e9
    # counter summaries are named by workload; the n = 3/2 power law has its own
    stem = "powerlaw-n1.5-" if args.workload == "powerlaw" and args.pl_n != 0.5 else args.workload
    traffic = measured_traffic(stem, args.n, choice)

    cpu = None
    if args.cpu_steps > 0:
        v, el = cpu_baseline(prob, args.cpu_steps)
        cpu = {"value": round(v, 4), "unit": "MLUPS", "cores": 1, "kind": "oracle",
               "sample": f"{args.cpu_steps} steps of the same {args.n}x{args.n} {args.workload} after 1 untimed step "
                         f"({el:.1f} s, single-threaded C oracle, -O2 -ffp-contract=off)"}

    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup + 5,
        "ms_per_step": gpu_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl,
                   "kernel": kname,
                   "partition": partition,
                   "autotuned": tuned,
                   "wall_s": round(wall, 4)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "algorithmic_bytes_per_launch": BYTES_PER_NODE * nodes},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    s.close()


def bench_batch(args):
    """256 periodic decaying-vortex instances (sizes 64..512, nu log-uniform in
    [1e-3, 1e-1], k^-3 fields, seed 20230614), one launch per step for all,
    replayed from a captured graph; MLUPS over the sum of all instances' nodes."""
    import torch

    from paper_2306_08216_amd import problems as P
    from paper_2306_08216_amd.batch import BatchSolver

    inst = P.batch_instances(256, seed=20230614)
    log("generating 256 instance fields")
    probs = [P.random_vortex(n, sd, nu) for n, nu, sd in inst]
    b = BatchSolver(probs)
    choice, cached = b.autotune(args.tuning, steps=10, retune=args.retune)
    nodes = b.nodes
    steps = min(args.steps, 500)
    b.step(min(args.warmup, 50))
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(b.stream)
    b.step_graph(steps)
    ev1.record(b.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    if args.copy_calib > 0:
        # known-size copies (k_pack, 80 B read + 80 B written per node) of the
        # largest instances, the reference for the byte counters
        big = sorted(range(b.count), key=lambda i: -probs[i].nodes)[:args.copy_calib]
        for i in big:
            b.save(i)
        torch.cuda.synchronize()
    mlups = nodes * steps / (ms / 1e3) / 1e6
    achieved = BYTES_PER_NODE * nodes / (ms / 1e3 / steps) / 1e9
    out = {
        "metric": METRIC, "value": round(mlups, 2), "unit": "MLUPS", "n_gpus": 1, "steps": steps,
        "warmup": min(args.warmup, 50), "ms_per_step": ms / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"batch of 256 periodic decaying vortices, sizes 64..512, {nodes} nodes, FP64",
                   "kernel": {1: "k_fused_batch", 2: "k_fused2_batch"}[choice[0]],
                   "autotuned": {"variant": choice[0], "tile_w": choice[3], "prefetch": choice[1], "rounds": choice[2],
                                 "from_cache": cached},
                   "workgroups": b.workgroups, "graph": True, "wall_s": round(wall, 4)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_batch_traffic(choice),
                     "algorithmic_bytes_per_launch": BYTES_PER_NODE * nodes},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    b.close()


if __name__ == "__main__":
    main()

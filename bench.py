"""Benchmark: block CG (blockCGrQ) vs N independent CG solves on one MI355X.

Workload (default): the 16^4 improved staggered operator (Gaussian fat links,
Haar long links), m = 0.05, N = 16 Gaussian right-hand sides, FP64 storage,
relative residual 1e-10 on every column.  One step is one complete block solve
of the 16-column block (initial CholQR, all iterations, reliable updates and
the final FP64 true-residual check), with inputs already resident in HBM.

Printed: ONE JSON line with the metric (solve time per right-hand side, lower
is better), the CG-baseline time per right-hand side on the same operator and
tolerance, the roofline of the dominant kernel (algorithmic bytes over its
average launch time, from HIP start / stop events carried by each hop dispatch on
the solver's stream), and the
CPU oracle timed on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solve time per RHS (block CG vs N× CG) at fixed residual; Dslash GB/s % HBM"
HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_1710_09745_amd", "csrc")

# Algorithmic bytes per even (or odd) site of one launch with N right-hand sides:
# every link and every vector element moved once.  vc = bytes per stored complex
# vector component (16-bit formats include their FP32 scale per 3 components),
# lm = bytes per stored folded link matrix (16 per site).
#   hop_oe : 16 link matrices + read P, write T              (6 N components)
#   hop_eo : 16 link matrices + read T, read P, write AP     (9 N components)
#   gram   : read both block vectors (6 N), or one when they alias (3 N)
#   pass_a : read Q, AP, write Q                             (9 N components)
#   pass_b : read Qt, P, write Q, P (12 N) + read and write the FP64 X (6 N x 16 B)
VC = {"fp64": 16.0, "fp32": 8.0, "fp16": 4.0 + 4.0 / 3.0, "bf16": 4.0 + 4.0 / 3.0, "fix16": 4.0 + 4.0 / 3.0}
LM = {"fp64": 144.0, "fp32": 72.0, "fp16": 40.0, "bf16": 40.0, "fix16": 40.0}


def model_bytes_per_site(kernel, N, prec="fp64", nl=16, aliased_gram=None):
    vc, link = VC[prec], nl * LM[prec]
    if kernel == "hop_oe":
        return link + 6 * N * vc
    if kernel == "hop_eo":
        return link + 9 * N * vc
    if kernel == "gram":
        return 3 * N * vc if aliased_gram else 6 * N * vc
    if kernel == "pass_a":
        return 9 * N * vc
    if kernel == "pass_b":
        return 12 * N * vc + 6 * N * 16
    return None


# source file of each timed kernel; its counters also depend on the shared headers
# and on the host code that picks its launch shape
KERNEL_SOURCE = {"hop_oe": "hop.hip", "hop_eo": "hop.hip", "pass_a": "blas.hip", "pass_b": "blas.hip",
                 "gram": "blas.hip"}


def kernel_source_hash(kernel):
    h = hashlib.sha256()
    files = sorted(f for f in os.listdir(CSRC) if f.endswith(".h")) + [KERNEL_SOURCE[kernel], "bcg_api.cpp"]
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel, workload_key, launch_bytes):
    """HBM bytes per launch from committed rocprofv3 --pmc summaries (FETCH_SIZE and
    WRITE_SIZE in KiB per dispatch, scaled by the copy-kernel calibration), or None
    when absent or taken on a different kernel source."""
    path = os.path.join(PROFILES, f"{kernel}_{workload_key}_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != kernel_source_hash(kernel):
        return None
    return float(d["hbm_bytes_per_launch"])


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


class Progress:
    """Prints the solver's progress to stderr at most every `every` seconds."""

    def __init__(self, label, every=10.0):
        self.label, self.every, self.last = label, every, time.perf_counter()

    def __call__(self, iters, rus, relres):
        now = time.perf_counter()
        if now - self.last >= self.every:
            self.last = now
            print(f"[bench] {self.label}: {iters} iterations, {rus} reliable updates, max rel res {relres:.2e}",
                  file=sys.stderr, flush=True)


def kernel_rates(ctx, bcg, N, prec, Vh):
    """Per-kernel average launch time (HIP events on the solver's stream) and
    algorithmic GB/s of the block iteration, from the kernel timers of the last solve."""
    rows = {}
    for k in ("hop_oe", "hop_eo", "pass_a", "pass_b", "gram"):
        n, ms = ctx.kernel_time(k)
        if not n:
            continue
        t = ms / n
        if k == "gram":
            # one non-aliased (P^H AP) and one aliased (Qt^H Qt) Gram per iteration
            b = 0.5 * (model_bytes_per_site(k, N, prec) + model_bytes_per_site(k, N, prec, aliased_gram=True)) * Vh
        else:
            b = model_bytes_per_site(k, N, prec) * Vh
        rows[k] = {"us": round(t * 1e3, 1), "launches": n, "bytes_per_launch": b,
                   "GB/s": round(b / (t * 1e-3) / 1e9, 1), "frac_hbm": round(b / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cg-steps", type=int, default=1)
    ap.add_argument("--cg-fp64", action="store_true",
                    help="with reduced storage, also time the FP64-storage CG baseline")
    ap.add_argument("--no-hbm-leg", action="store_true",
                    help="skip the 32^3x64 leg (kernel rooflines at HBM scale, oracle iteration time)")
    ap.add_argument("--hbm-iters", type=int, default=6)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", choices=["config2", "config3", "tsm192"], default="config2",
                    help="config2: 16^4, N=16, FP64 (default); config3: 32^3x64, FP32 + FP64 "
                         "reliable updates, tol 1e-8, N from --nrhs; tsm192: the paper's measurement "
                         "workload, 192 diluted noise sources solved at 5e-6 and 2e-9 in blocks of "
                         "--tsm-blocks (1 = the CG baseline)")
    ap.add_argument("--tsm-lattice", default="16x16x16x48")
    ap.add_argument("--tsm-mass", type=float, default=0.05)
    ap.add_argument("--tsm-blocks", default="1,8,16,24,32,48,64")
    ap.add_argument("--tsm-links", choices=["random", "smooth"], default="random",
                    help="tsm192 links: Gaussian fat + Haar long (random), or smooth SU(3) exp(i eps H) "
                         "fields standing in for smeared ensembles (smooth)")
    ap.add_argument("--tsm-eps", type=float, default=0.6, help="eps of the smooth links")
    ap.add_argument("--tsm-pseudo", action="store_true",
                    help="tsm192: also run pseudo-block CG at every block size > 1 (FP64 storage)")
    ap.add_argument("--sstep", default="2,4",
                    help="also time s-step block CG at these s (FP64 storage, comma list; '' = none)")
    ap.add_argument("--nrhs", type=int, default=16)
    ap.add_argument("--prec", default=None, help="storage precision override (fp64/fp32/fp16/bf16/fix16)")
    ap.add_argument("--no-cg", action="store_true")
    ap.add_argument("--sweep", default=None,
                    help="comma-separated N list: per-kernel GB/s of the 32^3x64 block iteration vs N "
                         "(a few iterations per N, FP32 storage unless --prec), one JSON line")
    ap.add_argument("--sweep-iters", type=int, default=5)
    ap.add_argument("--sweep-lattice", default="32x32x32x64", choices=["32x32x32x64", "16x16x16x16"])
    ap.add_argument("--hop-opts", default=None,
                    help="launch options for the sweep, e.g. hop_kernel=2,hop_tr=8,hop_tpb=1")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB device to device three times (the reference kernel for "
                         "scaling rocprofv3 FETCH_SIZE / WRITE_SIZE to HBM bytes)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the solver runs on one GPU; the multi-GPU path (right-hand-side blocks "
              "per GPU, or lattice domain decomposition) is a design only. Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1710_09745_amd import bcg, synth

    if args.copy_calibration:
        copy_calibration(torch)
    if args.sweep:
        return sweep(args, bcg, synth, torch)
    if args.workload == "tsm192":
        return tsm192(args, bcg, synth, torch)

    if args.workload == "config2":
        c = synth.CONFIGS[2]
        dims, m, N, tol, prec = c["dims"], c["mass"], c["nrhs"], c["tol"], "fp64"
        fat, lng, B = synth.config_inputs(2)
    else:
        c = synth.CONFIGS[3]
        dims, m, N, tol, prec = c["dims"], c["mass"], args.nrhs, c["tol"], "fp32"
        fat, lng, B = synth.config_inputs(3, nrhs=N)
    if args.prec:
        prec = args.prec
    wkey = f"{'x'.join(str(d) for d in dims)}_n{N}_{prec}"
    workload = (f"{'x'.join(str(d) for d in dims)} improved staggered (fat N(0,1)/3 + Haar long), "
                f"m={m}, N={N}, {prec} storage{' + FP64 reliable updates' if prec != 'fp64' else ''}, "
                f"tol {tol:g}")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ctx = bcg.Context(dims, improved=True, device=dev)
    ctx.load_links(fat, lng)
    ctx.set_mass(m)
    ctx.set_solver(tol=tol, max_iter=100000, prec=prec, ru_delta=0.1)
    ctx.set_monitor(Progress("block solve"))
    Bt = torch.from_numpy(B).to(dev)
    torch.cuda.synchronize()
    print(f"[bench] workload: {workload}", file=sys.stderr, flush=True)

    # warmup, with every kernel class timed to find the dominant one
    ctx.set_profiling(bcg.KERNELS)
    ctx.profile_reset()
    info = None
    for _ in range(max(1, args.warmup)):
        X, info = ctx.solve(Bt)
    torch.cuda.synchronize()
    breakdown = {}
    for k in bcg.KERNELS:
        n, ms = ctx.kernel_time(k)
        if n:
            breakdown[k] = {"launches": n, "total_ms": ms}
    dominant = max((k for k in breakdown if model_bytes_per_site(k, N) is not None),
                   key=lambda k: breakdown[k]["total_ms"])
    print(f"[bench] warmup solve: iters={info['iters']} rus={info['reliable_updates']} "
          f"max true rel res={info['max_true_rel_res']:.2e}; dominant kernel {dominant}",
          file=sys.stderr, flush=True)

    # timed region: K block solves; only the dominant kernel is timed by events
    ctx.set_profiling([dominant])
    ctx.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    for _ in range(args.steps):
        X, info = ctx.solve(Bt)
        iters.append(info["iters"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    launches, kms = ctx.kernel_time(dominant)
    ctx.set_profiling([])
    max_res = info["max_true_rel_res"]

    # CG baseline: N independent FP64 solves, same operator and tolerance
    # CG baseline: N independent solves, same operator, tolerance and storage precision
    # (double-single CG with reliable updates when the storage is not FP64)
    cg_ms, ic = None, None
    cg64_ms, ic64 = None, None
    if not args.no_cg:
        ctx.set_monitor(Progress("CG baseline"))

        def time_cg(p):
            ctx.set_solver(tol=tol, max_iter=100000, prec=p, ru_delta=0.1)
            _, i0 = ctx.solve_cg(Bt)      # warm
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            for _ in range(args.cg_steps):
                _, i0 = ctx.solve_cg(Bt)
            torch.cuda.synchronize()
            return (time.perf_counter() - t2) * 1e3 / args.cg_steps, i0

        cg_ms, ic = time_cg(prec)
        if prec != "fp64" and args.cg_fp64:
            cg64_ms, ic64 = time_cg("fp64")
        ctx.set_solver(tol=tol, max_iter=100000, prec=prec, ru_delta=0.1)
        print(f"[bench] block {ms_per_step:.2f} ms/solve ({iters[-1]} iters), CG ({prec}) {cg_ms:.2f} ms "
              f"for {N} columns ({ic['iters']} iters)", file=sys.stderr, flush=True)
    # pseudo-block CG (N independent recurrences sharing each stencil application, FP64):
    # CG -> pseudo-block is the gain of sharing the links, pseudo-block -> block CG the
    # gain of sharing the Krylov space
    pb_ms, ipb = None, None
    if not args.no_cg and prec == "fp64":
        ctx.set_monitor(Progress("pseudo-block CG"))
        _, ipb = ctx.solve_pseudo(Bt)      # warm
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for _ in range(args.cg_steps):
            _, ipb = ctx.solve_pseudo(Bt)
        torch.cuda.synchronize()
        pb_ms = (time.perf_counter() - t2) * 1e3 / args.cg_steps
        print(f"[bench] pseudo-block {pb_ms:.2f} ms for {N} columns ({ipb['iters']} lockstep iters)",
              file=sys.stderr, flush=True)

    # s-step block CG (FP64, or FP32 storage with reliable updates): s block
    # directions per outer iteration, one reduction phase per outer iteration
    # instead of two per iteration
    sstep = []
    if prec in ("fp64", "fp32") and args.sstep:
        for sv in [int(x) for x in args.sstep.split(",") if x.strip()]:
            if sv * N > 64:
                continue
            ctx.set_monitor(Progress(f"s-step s={sv}"))
            _, iss = ctx.solve_sstep(Bt, sv)      # warm (and the library's spectrum estimate)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            for _ in range(args.cg_steps):
                _, iss = ctx.solve_sstep(Bt, sv)
            torch.cuda.synchronize()
            ss_ms = (time.perf_counter() - t3) * 1e3 / args.cg_steps
            sstep.append({"s": sv, "ms_per_rhs": round(ss_ms / N, 4), "steps": iss["iters"],
                          "restarts": iss["restarts"], "reliable_updates": iss["reliable_updates"],
                          "max_true_rel_res": iss["max_true_rel_res"],
                          "us_per_step": round(ss_ms / max(iss["iters"], 1) * 1e3, 1)})
            print(f"[bench] s-step s={sv}: {ss_ms:.2f} ms for {N} columns ({iss['iters']} steps)",
                  file=sys.stderr, flush=True)

    # roofline of the dominant kernel
    Vh = synth.volume(dims) // 2
    per_site = model_bytes_per_site(dominant, N, prec)
    launch_bytes = per_site * Vh
    avg_ms = kms / max(launches, 1)
    achieved = launch_bytes / (avg_ms * 1e-3) / 1e9
    traffic = load_traffic(dominant, wkey, launch_bytes)
    roofline = {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "bytes_per_launch": launch_bytes,
                "avg_launch_ms": round(avg_ms, 5), "launches": launches}
    dslash = {}
    for k in ("hop_oe", "hop_eo"):
        if k in breakdown:
            b = model_bytes_per_site(k, N, prec) * Vh
            t = breakdown[k]["total_ms"] / breakdown[k]["launches"]
            dslash[k] = {"GB/s": round(b / (t * 1e-3) / 1e9, 1),
                         "frac_hbm": round(b / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(dims, fat, lng, m, B, tol, iters[-1], args.cpu_seconds)
    ctx.close()
    del Bt
    hbm = None
    if not args.no_hbm_leg and args.workload == "config2":
        hbm = hbm_leg(args, bcg, synth, torch, dev)

    out = {
        "metric": METRIC,
        "value": round(ms_per_step / N, 4),
        "unit": "ms/RHS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32+f64", "fp16": "f16+f64", "bf16": "bf16+f64",
                  "fix16": "i16+f32+f64"}[prec],
        "data": "synthetic",
        "config": {"workload": workload, "lattice": list(dims), "nrhs": N, "mass": m,
                   "tol": tol, "storage": prec, "parallelism": "single GPU"},
        "block_iters": iters[-1],
        "block_reliable_updates": info["reliable_updates"],
        "block_max_true_rel_res": max_res,
        "cg_storage": prec,
        "cg_ms_per_rhs": round(cg_ms / N, 4) if cg_ms else None,
        "cg_iters_per_rhs": round(ic["iters"] / N, 1) if ic else None,
        "cg_max_true_rel_res": ic["max_true_rel_res"] if ic else None,
        "speedup_vs_cg": round(cg_ms / ms_per_step, 3) if cg_ms else None,
        "pseudo_block_ms_per_rhs": round(pb_ms / N, 4) if pb_ms else None,
        "pseudo_block_iters": ipb["iters"] if ipb else None,
        "speedup_link_reuse": round(cg_ms / pb_ms, 3) if (pb_ms and cg_ms) else None,
        "speedup_krylov_sharing": round(pb_ms / ms_per_step, 3) if pb_ms else None,
        "sstep": sstep or None,
        "cg_fp64_ms_per_rhs": round(cg64_ms / N, 4) if cg64_ms else None,
        "speedup_vs_cg_fp64": round(cg64_ms / ms_per_step, 3) if cg64_ms else None,
        "roofline": roofline,
        "dslash": dslash,
        "kernel_breakdown_warmup_ms": {k: round(v["total_ms"], 3) for k, v in breakdown.items()},
        "cpu_baseline": cpu,
        "hbm_leg": hbm,
    }
    print(json.dumps(out), flush=True)


def sweep(args, bcg, synth, torch):
    """Kernel GB/s of the block iteration vs N on the 32^3x64 lattice (or the 16^4
    one with --sweep-lattice 16x16x16x16): each N runs a fixed number of block
    iterations (reliable updates off, so every iteration does the same work) with
    every kernel class timed by HIP events.  --hop-opts sets launch options."""
    cfg = 2 if args.sweep_lattice == "16x16x16x16" else 3
    c = synth.CONFIGS[cfg]
    dims, m = c["dims"], c["mass"]
    prec = args.prec or ("fp32" if cfg == 3 else "fp64")
    fat, lng, _ = synth.config_inputs(cfg, nrhs=1)
    Vh = synth.volume(dims) // 2
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ctx = bcg.Context(dims, improved=True, device=dev)
    ctx.load_links(fat, lng)
    ctx.set_mass(m)
    opts = {}
    for kv in (args.hop_opts.split(",") if args.hop_opts else []):
        k, v = kv.split("=")
        opts[k] = int(v)
        ctx.set_option(k, int(v))
    rows = []
    for N in [int(x) for x in args.sweep.split(",")]:
        B = synth.rhs(synth.make_rng(7), N, dims)
        Bt = torch.from_numpy(B).to(dev)
        ctx.set_solver(tol=1e-14, max_iter=args.sweep_iters, prec=prec, ru_delta=0.0)
        ctx.set_stability(ru_window=0, stall_limit=0)
        ctx.solve(Bt, raise_on_error=False)                      # warm (buffers, links)
        ctx.set_profiling(bcg.KERNELS)
        ctx.profile_reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.solve(Bt, raise_on_error=False)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ctx.set_profiling([])
        row = {"nrhs": N, "iters": args.sweep_iters, "solve_ms": round(wall * 1e3, 3)}
        for k, v in kernel_rates(ctx, bcg, N, prec, Vh).items():
            row[k] = {kk: v[kk] for kk in ("us", "GB/s", "frac_hbm")}
        rows.append(row)
        print(f"[sweep] N={N}: " + json.dumps(row), file=sys.stderr, flush=True)
        del Bt
    print(json.dumps({"metric": f"block-iteration kernel GB/s vs N ({'x'.join(str(d) for d in dims)} improved "
                                f"staggered)", "storage": prec, "dims": list(dims), "options": opts, "rows": rows}),
          flush=True)
    ctx.close()


def tsm192(args, bcg, synth, torch):
    """The paper's measurement workload (Sec. 7.1) on synthetic links: 192 right-hand
    sides (24 noise sources x 8 disjoint-support subsets), every one solved twice as in
    the truncated solver method, to 5e-6 (sloppy) and to 2e-9 (fine), in blocks of b
    consecutive sources (b = 1: one CG solve per source, the baseline).  Prints one
    JSON line: total time, iterations and worst true residual per block size (the
    analogue of the paper's time-to-solution and iteration-count figures)."""
    dims = tuple(int(x) for x in args.tsm_lattice.split("x"))
    m = args.tsm_mass
    prec = args.prec or "fp64"
    blocks = [int(b) for b in args.tsm_blocks.split(",")]
    if args.tsm_links == "smooth":
        fat, lng = synth.smooth_links(synth.make_rng(synth.seed_for(6, 4)), dims, args.tsm_eps)
    else:
        fat = synth.fat_links(synth.make_rng(synth.seed_for(6, 0)), dims)
        lng = synth.long_links(synth.make_rng(synth.seed_for(6, 0) + 1), dims)
    B = synth.diluted_noise_sources(dims, 24, 8, synth.make_rng(synth.seed_for(6, 1)))
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ctx = bcg.Context(dims, improved=True, device=dev)
    ctx.load_links(fat, lng)
    ctx.set_mass(m)
    Bt = torch.from_numpy(B).to(dev)
    total = Bt.shape[0]

    def solve_all(kind, b):
        """Every source solved to 5e-6 and to 2e-9 with one method in blocks of b."""
        out = {}
        for name, tol in (("sloppy", 5e-6), ("fine", 2e-9)):
            ctx.set_solver(tol=tol, max_iter=100000, prec=prec, ru_delta=0.1)
            ctx.set_monitor(Progress(f"tsm192 {kind} b={b} {name}"))
            call = {"cg": ctx.solve_cg, "block": ctx.solve, "pseudo": ctx.solve_pseudo}[kind]
            call(Bt[:b].contiguous(), raise_on_error=False)          # warm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            its = rhs_its = 0
            worst = 0.0
            fails = 0
            for j in range(0, total, b):
                _, info = call(Bt[j:j + b].contiguous(), raise_on_error=False)
                its += info["iters"]
                # block and pseudo-block: one iteration applies A to all b columns; CG runs
                # its columns in turn and reports their summed iterations
                rhs_its += info["iters"] if kind == "cg" else info["iters"] * b
                worst = max(worst, info["max_true_rel_res"])
                fails += info["rc"] != 0
            torch.cuda.synchronize()
            out[name] = {"ms": round((time.perf_counter() - t0) * 1e3, 1), "iters": its, "rhs_iters": rhs_its,
                         "max_true_rel_res": worst, "failed_solves": fails}
        out["total_ms"] = round(out["sloppy"]["ms"] + out["fine"]["ms"], 1)
        return out

    rows = []
    for b in blocks:
        if total % b:
            continue
        row = {"block": b, "solves": total // b}
        row.update(solve_all("cg" if b == 1 else "block", b))
        if b > 1 and args.tsm_pseudo and prec == "fp64":
            row["pseudo"] = solve_all("pseudo", b)
        rows.append(row)
        print(f"[tsm192] b={b}: {row['total_ms']} ms (sloppy {row['sloppy']['iters']} + fine "
              f"{row['fine']['iters']} iterations)"
              + (f"; pseudo-block {row['pseudo']['total_ms']} ms" if "pseudo" in row else ""),
              file=sys.stderr, flush=True)
    base = next((r["total_ms"] for r in rows if r["block"] == 1), None)
    for r in rows:
        r["speedup_vs_cg"] = round(base / r["total_ms"], 3) if base else None
    links = ("Gaussian fat + Haar long" if args.tsm_links == "random"
             else f"smooth SU(3) exp(i eps H), eps={args.tsm_eps}")
    print(json.dumps({"metric": "total time for 192 diluted sources, sloppy 5e-6 + fine 2e-9, vs block size",
                      "lattice": list(dims), "mass": m, "storage": prec, "links": links, "data": "synthetic",
                      "rows": rows}), flush=True)
    ctx.close()


def copy_calibration(torch):
    """Three 1 GiB device-to-device copies: the reference kernel for scaling the
    rocprofv3 FETCH_SIZE / WRITE_SIZE counters to bytes of HBM traffic."""
    dev = torch.device("cuda:0")
    a = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    print("[bench] copy calibration: 3 x 1 GiB device copies", file=sys.stderr, flush=True)


def hbm_leg(args, bcg, synth, torch, dev, N=16, prec="fp32"):
    """Rooflines at HBM scale: a fixed number of block iterations on the 32^3 x 64
    lattice (N = 16, FP32 storage; its working set is far beyond the 256 MB
    Infinity Cache), every kernel timed with HIP events on the solver's stream,
    reliable updates off so that every iteration does the same work; next to it
    the oracle's time per block iteration on the same input (two iterations)."""
    c = synth.CONFIGS[3]
    dims, m = c["dims"], c["mass"]
    Vh = synth.volume(dims) // 2
    t0 = time.perf_counter()
    fat, lng, B = synth.config_inputs(3, nrhs=N)
    print(f"[bench] hbm leg: 32^3x64 inputs drawn in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    ctx = bcg.Context(dims, improved=True, device=dev)
    ctx.load_links(fat, lng)
    ctx.set_mass(m)
    ctx.set_solver(tol=1e-14, max_iter=args.hbm_iters, prec=prec, ru_delta=0.0)
    ctx.set_stability(ru_window=0, stall_limit=0)
    Bt = torch.from_numpy(B).to(dev)
    ctx.solve(Bt, raise_on_error=False)                      # warm (buffers, sloppy links)
    ctx.set_profiling(bcg.KERNELS)
    ctx.profile_reset()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.solve(Bt, raise_on_error=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    rows = kernel_rates(ctx, bcg, N, prec, Vh)
    ctx.set_profiling([])
    ctx.close()
    del Bt
    dominant = max(rows, key=lambda k: rows[k]["us"] * rows[k]["launches"])
    d = rows[dominant]
    wkey = f"{'x'.join(str(x) for x in dims)}_n{N}_{prec}"
    roof = {"bound": "hbm", "kernel": dominant, "achieved": d["GB/s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": d["frac_hbm"], "traffic": load_traffic(dominant, wkey, d["bytes_per_launch"]),
            "bytes_per_launch": d["bytes_per_launch"], "avg_launch_ms": round(d["us"] * 1e-3, 5),
            "launches": d["launches"]}
    print(f"[bench] hbm leg: {args.hbm_iters} iterations in {wall * 1e3:.1f} ms; dominant {dominant} "
          f"{d['GB/s']} GB/s", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu:
        import oracle
        op = oracle.Operator(dims, fat, lng, m)
        k = 2
        t2 = time.perf_counter()
        oracle.block_cg_rq(op.apply, B, 1e-30, max_iter=k)
        t = time.perf_counter() - t2
        cpu = {"value": round(t / k * 1e3, 1), "unit": "ms per block iteration", "cores": oracle.num_threads(),
               "cpu": cpu_model(), "kind": "oracle",
               "sample": f"oracle blockCGrQ (FP64) on the same 32x32x32x64 N={N} input, {k} iterations "
                         f"(initial CholQR included) in {t:.1f} s"}
        print(f"[bench] hbm leg: oracle {t / k:.2f} s per block iteration", file=sys.stderr, flush=True)
    return {"workload": f"32x32x32x64 improved staggered, m={m}, N={N}, {prec} storage, "
                        f"{args.hbm_iters} block iterations without reliable updates",
            "ms_per_iteration": round(wall * 1e3 / args.hbm_iters, 3),
            "roofline_hbm": roof, "kernels": {k: {kk: v[kk] for kk in ("us", "GB/s", "frac_hbm")}
                                              for k, v in rows.items()},
            "cpu_oracle": cpu}


def cpu_baseline(dims, fat, lng, m, B, tol, gpu_iters, budget_s):
    """The oracle's blockCGrQ on the same input, run for a bounded number of
    iterations and extrapolated to the GPU's iteration count."""
    import oracle

    op = oracle.Operator(dims, fat, lng, m)
    t0 = time.perf_counter()
    oracle.block_cg_rq(op.apply, B, 1e-30, max_iter=2)
    t_probe = (time.perf_counter() - t0) / 2
    k = max(2, min(gpu_iters, int(budget_s / max(t_probe, 1e-6))))
    t0 = time.perf_counter()
    oracle.block_cg_rq(op.apply, B, 1e-30, max_iter=k)
    t = time.perf_counter() - t0
    per_iter = t / k
    N = B.shape[0]
    est = per_iter * gpu_iters
    return {"value": round(est * 1e3 / N, 2), "unit": "ms/RHS", "cores": oracle.num_threads(),
            "cpu": cpu_model(), "kind": "oracle",
            "sample": f"oracle blockCGrQ (C stencil + NumPy) on the same {'x'.join(str(d) for d in dims)} "
                      f"N={N} input, first {k} iterations in {t:.1f} s, extrapolated to the GPU's "
                      f"{gpu_iters} iterations"}


if __name__ == "__main__":
    main()

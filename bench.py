"""Benchmark: cell-updates per second per SSP-RK3 stage of the MR blast workload
(3 levels, 128^3 effective, 16^3 blocks + 4 halo layers), FP32 batched path, one MI355X.

One "step" is one global time step of the whole hot path: CFL reduction, three stages of
{restriction, halo fill, fused right-hand side + stage update, jump correction}, then the
MR adaptation (restriction, 26-region halo fill, details/flags, flag read-back, tree
update, prediction of new children).  value = (leaf cells x 3 stages) summed over the timed
steps / wall time, with the state resident in HBM.

Also measured on the same workload: the FP64 plain path (speed-up), the L1 density
difference and flag agreement between the two GPU paths, the dominant kernel's average
duration from HIP events (roofline), and the FP64 CPU oracle on a bounded sample.
Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FLOPs of the fused right-hand side + update per cell-update, counted from the
# textbook formulation: per face 734 FLOPs with every characteristic field upwind (17 for the
# new cell's primitives, 40 for the Roe average and eigen-quantities, 234 for projecting six
# cells' states and fluxes, 66 to assemble the fields, 22 for the back-projection, 5 for the
# difference, 70 per WENO5), plus 110 per field that takes the LLF split; 17/16 faces per
# cell per axis; 40 per cell for the update.
FACE_BASE, LLF_EXTRA, UPDATE = 734.0, 110.0, 40.0
PEAK_FP32_VECTOR = 157.3e12       # MI355X FP32 vector (FLOP/s)
PEAK_HBM = 8.0e12                 # bytes/s


def counted_traffic(kernel: str):
    """HBM bytes per launch of the given fused-kernel variant from the committed counter
    summary, or None when the kernel source changed since the counters were taken."""
    import hashlib
    try:
        prof = json.load(open(os.path.join(ROOT, "profiles", "rhs_update_blast128_counters.json")))
        src = open(os.path.join(ROOT, prof["source"]), "rb").read()
    except (OSError, KeyError, ValueError):
        return None
    if hashlib.sha256(src).hexdigest()[:16] != prof["source_sha256_16"]:
        return None
    return prof.get("traffic_bytes_per_dispatch", {}).get(kernel)


def kernel_name(shape) -> str:
    """Demangled name of the fused kernel's instantiation for a variant shape."""
    gp, tpb, wpe = shape
    b = lambda v: "true" if v else "false"
    return f"k_rhs_update<float, {gp}, {abs(tpb)}, {b(tpb < 0)}, {wpe}>"


def flops_per_cell_update(llf_fraction: float) -> float:
    return 3.0 * (17.0 / 16.0) * (FACE_BASE + 5.0 * llf_fraction * LLF_EXTRA) + UPDATE


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_gpu(pb, dtype, batched, warmup, steps, timing=False, variant=None):
    """Timed run of `steps` steps through the library's own step loop (mrfv_run).  The
    batched FP32 path autotunes the fused kernel's launch shape after the warm-up (or
    takes `variant`)."""
    import torch
    from paper_2012_04385_amd.mrfv import Solver
    g = Solver([pb], dtype=dtype, batched=batched).init()
    for _ in range(warmup):
        g.step()
    g.check()
    g.tuned = None
    if batched and dtype == "f32":
        if variant is None:
            choice, ms = g.autotune(reps=5)
            g.tuned = {"choice": choice, "shapes": g.rhs_variants(), "ms_per_launch": ms}
            log(f"[bench] autotune: variant {choice} {g.rhs_variants()[choice]} "
                f"(ms per launch: {', '.join(f'{m:.3f}' for m in ms)})")
        else:
            g.set_rhs_variant(variant)
    if timing:
        g.enable_kernel_timing(True)
        g.kernel_time()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cells = 3 * g.run(steps)     # the library's step loop; leaf cells of every step's tree
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g.check()
    kt = g.kernel_time() if timing else None
    return g, cells, t1 - t0, kt


def run_trees(pb, dtype, batched, steps):
    """Untimed run recording the leaf set after every step (flag agreement)."""
    from paper_2012_04385_amd.mrfv import Solver
    g = Solver([pb], dtype=dtype, batched=batched).init()
    trees = []
    for _ in range(steps):
        g.step()
        info = g.blocks()
        trees.append(frozenset(tuple(int(v) for v in r[2:6]) for r in info if r[6] == 1))
    g.check()
    return g, trees


def cpu_baseline(pb, budget_s=15.0, max_steps=10):
    from oracle import oracle
    o = oracle.Sim(pb).init()
    cells, n, llf = 0, 0, []
    t0 = time.perf_counter()
    while n < max_steps and (time.perf_counter() - t0) < budget_s:
        leaves = int((o.blocks()[:, 4] == 1).sum())
        o.step()
        llf.append(o.llf_fraction)
        cells += leaves * 16 ** 3 * 3
        n += 1
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": cells / dt, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n} of {pb.steps} steps of {pb.name} (FP64, OpenMP over blocks)"}, \
        sum(llf) / len(llf)


def other_workload(args):
    """Throughput of the FP32 batched path (step graph, autotuned shape) on a larger
    workload; the fused kernel's duration from HIP events on an eager run."""
    import torch
    from paper_2012_04385_amd import workloads as W
    from paper_2012_04385_amd.mrfv import Solver
    pbs = {"kh_256e_5lvl": lambda: [W.kh_mr5(steps=args.warmup + args.steps)],
           "multi_256": lambda: W.multi_instance(steps=args.warmup + args.steps),
           "shockblobs_512e_6lvl": lambda: [W.shock_blobs_mr6(steps=args.warmup + args.steps)]}[args.workload]()
    res = {}
    for batched, timing in ((2, False), (1, True)):
        g = Solver(pbs, dtype="f32", batched=batched).init()
        for _ in range(args.warmup):
            g.step()
        g.check()
        if batched == 2:
            choice, ms = g.autotune(reps=3)
            res["autotune"] = {"choice": choice, "shapes": g.rhs_variants(), "ms_per_launch": ms}
        else:
            g.set_rhs_variant(res["autotune"]["choice"])
            g.enable_kernel_timing(True)
            g.kernel_time()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cells = 3 * g.run(args.steps)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        g.check()
        # MR compression: leaf cells over the cells of the uniform finest grid
        full = sum(pb.n0[0] * pb.n0[1] * pb.n0[2] * 8 ** pb.lmax * 16 ** 3 for pb in pbs)
        res[batched] = (cells / secs, 1e3 * secs / args.steps, g.kernel_time() if timing else None,
                        g.stats()[1], g.step_timing(), g.stats()[2] / full)
        log(f"[bench] {args.workload} batched={batched}: {res[batched][0]:.4e} cell-updates/s, "
            f"{res[batched][1]:.2f} ms/step")
        del g
        torch.cuda.empty_cache()
    launches, total_ms, kcells = res[1][2]
    avg_s = total_ms / 1e3 / max(launches, 1)
    kname = kernel_name(res["autotune"]["shapes"][res["autotune"]["choice"]])
    fpc = flops_per_cell_update(0.5)
    achieved = kcells / max(launches, 1) * fpc / avg_s
    out = {"metric": "cell-updates/s per RK stage (FP32 batched MR RK3)", "value": res[2][0],
           "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": res[2][1], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": args.workload, "instances": len(pbs), "leaves_final": res[2][3],
                      "compression": res[2][5],
                      "path": "batched FP32, steps replayed from a hipGraph, next step queued ahead"},
           "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VECTOR / 1e12,
                        "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR, "traffic": None,
                        "kernel": kname,
                        "avg_launch_ms": avg_s * 1e3,
                        "flop_model_llf_fraction": 0.5},
           "cpu_baseline": None, "value_eager_launches": res[1][0], "autotune": res["autotune"],
           "host_adaptation_ms_per_step": {k: v / max(res[2][4]["steps"], 1) for k, v in res[2][4].items()
                                           if k != "steps"}}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=45)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 plain comparison")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a device copy of 512 MiB (calibrates HBM byte counters)")
    ap.add_argument("--proposer-gain", action="store_true",
                    help="only run the learned-proposer gain test (6-level shock-blobs workload)")
    ap.add_argument("--workload", default="blast_128e_3lvl",
                    choices=["blast_128e_3lvl", "kh_256e_5lvl", "multi_256", "shockblobs_512e_6lvl"],
                    help="other workloads: FP32 batched throughput only (no FP64, no CPU leg)")
    args = ap.parse_args()
    if args.proposer_gain:
        from paper_2012_04385_amd.proposer import gain_test
        print(json.dumps(gain_test(log=log)), flush=True)
        return
    if args.copy_calibration:
        import torch
        src = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4,
                          "launches": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design note, not part of this build)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2012_04385_amd import workloads as W

    if args.workload != "blast_128e_3lvl":
        other_workload(args)
        return

    pb = W.blast_mr3(steps=args.warmup + args.steps)
    log(f"[bench] workload {pb.name}: FP32 batched, warmup {args.warmup}, timed {args.steps}")
    g32, cells, secs, _ = run_gpu(pb, "f32", 2, args.warmup, args.steps)
    value = cells / secs
    tuned = g32.tuned
    log(f"[bench] FP32 batched, stage hipGraph: {value:.4e} cell-updates/s, "
        f"{1e3 * secs / args.steps:.3f} ms/step")
    del g32
    # same steps with eager launches and HIP events around every fused-kernel launch
    ge, cells_e, secs_e, kt = run_gpu(pb, "f32", 1, args.warmup, args.steps, timing=True,
                                      variant=tuned["choice"])
    value_eager = cells_e / secs_e
    log(f"[bench] FP32 batched, eager + kernel events: {value_eager:.4e} cell-updates/s")
    del ge

    extra = {}
    if not args.no_fp64:
        log("[bench] FP64 plain path on the same workload")
        g64, cells64, secs64, _ = run_gpu(pb, "f64", False, args.warmup, args.steps)
        del g64
        v64 = cells64 / secs64
        log(f"[bench] FP64 plain: {v64:.4e} cell-updates/s")
        nsteps = args.warmup + args.steps
        a32, trees32 = run_trees(pb, "f32", True, nsteps)
        a64, trees64 = run_trees(pb, "f64", False, nsteps)
        s32, s64 = a32.leaf_states(), a64.leaf_states()
        common = set(s32) & set(s64)
        l1 = sum(np.abs(s32[k][0] - s64[k][0]).sum() * pb.dx(k[0]) ** 3 for k in common)
        same = sum(1 for a, b in zip(trees32, trees64) if a == b)
        extra = {"fp64_plain_value": v64, "speedup_vs_fp64_plain": value / v64,
                 "l1_rho_fp32_vs_fp64": l1, "steps_with_identical_flags": f"{same}/{nsteps}"}
        log(f"[bench] L1(rho) FP32 vs FP64 after {nsteps} steps = {l1:.3e}; identical trees "
            f"after {same}/{nsteps} steps")
        del a32, a64

    cpu, llf = None, 0.5
    if not args.no_cpu:
        log("[bench] CPU oracle sample")
        cpu, llf = cpu_baseline(W.blast_mr3(steps=args.warmup + args.steps))
        log(f"[bench] oracle: {cpu['value']:.4e} cell-updates/s on {cpu['cores']} threads; "
            f"LLF fraction {llf:.3f}")

    launches, total_ms, kcells = kt
    avg_s = total_ms / 1e3 / max(launches, 1)
    cells_per_launch = kcells / max(launches, 1)
    fpc = flops_per_cell_update(llf)
    achieved = cells_per_launch * fpc / avg_s
    kname = kernel_name(tuned["shapes"][tuned["choice"]])
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VECTOR / 1e12,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR, "traffic": counted_traffic(kname),
            "kernel": kname, "avg_launch_ms": avg_s * 1e3,
            "cells_per_launch": cells_per_launch, "flop_per_cell_update": fpc,
            "llf_fraction": llf}
    ms_step = 1e3 * secs / args.steps
    out = {"metric": "cell-updates/s per RK stage (FP32 batched MR RK3)", "value": value,
           "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": pb.name, "levels": pb.lmax + 1, "effective_grid": 128,
                      "block": "16^3 + 4 halo", "ic": "spherical blast r=0.1, (1,10)|(0.125,0.1), "
                      "+-1e-3 rho noise", "eps": pb.eps, "cfl": pb.cfl,
                      "path": "batched FP32, steps replayed from a hipGraph, next step queued ahead"},
           "roofline": roof, "cpu_baseline": cpu}
    out["value_eager_launches"] = value_eager
    out["autotune"] = tuned
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

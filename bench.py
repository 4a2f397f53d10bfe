"""Benchmark: cell-updates per second per SSP-RK3 stage of the FP32 batched MR path on one
MI355X.  Default workload: the 6-level shock-blobs problem (512^3 effective, 16^3 blocks +
4 halo layers, resolution jumps in every step), the largest single-GPU configuration.

One "step" is one global time step of the whole hot path: CFL reduction, three stages of
{restriction, halo fill, fused right-hand side + stage update, jump correction}, then the
MR adaptation (restriction, halo fill, details/flags, flag read-back, tree update,
prediction of new children).  value = (leaf cells x 3 stages) summed over the timed steps
/ wall time, with the state resident in HBM, steps run by the library's own step loop
(step graph replays, the next step queued before the flags are read).

Also measured on the same workload:
  * parity: the FP64 CPU oracle and the GPU run the first steps from the same seeded
    initial condition; identical leaf sets after algo:Init and every step, L1 density and
    energy differences at the end (volume-weighted, over the whole domain);
  * cpu_baseline: the oracle's rate on those steps (threads, physical cores, CPU model);
  * roofline: the fused kernel's average duration from HIP events around each launch on
    the library's stream (eager run with the autotuned shape), against the FP32 vector
    peak, plus its algorithmic HBM bandwidth and the counter-measured traffic;
  * the FP64 plain path on the same workload (speed-up), and config 2 (the 3-level blast)
    as extra keys.
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
PEAK_FP32_VECTOR = 157.3e12       # MI355X FP32 vector with packed FP32 (FLOP/s)
PEAK_FP32_UNPACKED = 78.6e12      # without packed FP32 instructions (compiled out here)
PEAK_FP64_VECTOR = 78.6e12        # MI355X FP64 vector (FLOP/s)
PEAK_HBM = 8.0e12                 # bytes/s
# algorithmic bytes per FP32 cell-update of the fused kernel, every stage: read the interior
# and the 3-wide face layers (5 components x 4 B x 8704 / 4096 cells = 42.5 B), write the new
# state (20 B), and write U0 (stage 1) or read it (stages 2, 3) (20 B)
BYTES_PER_CELL_UPDATE = 82.5

WORKLOADS = ["shockblobs_512e_6lvl", "blast_128e_3lvl", "kh_256e_5lvl", "multi_256", "localblast_256e_5lvl"]


def problems(name, steps):
    from paper_2012_04385_amd import workloads as W
    return {"shockblobs_512e_6lvl": lambda: [W.shock_blobs_mr6(steps=steps)],
            "blast_128e_3lvl": lambda: [W.blast_mr3(steps=steps)],
            "kh_256e_5lvl": lambda: [W.kh_mr5(steps=steps)],
            "multi_256": lambda: W.multi_instance(steps=steps),
            "localblast_256e_5lvl": lambda: [W.local_blast_mr5(steps=steps)]}[name]()


def describe(name, pbs):
    pb = pbs[0]
    ics = {"shockblobs_512e_6lvl": "Mach-2 shock at x=0.1 into 32 seeded Gaussian density blobs "
                                   "(amplitude 0.5, width 0.02)",
           "blast_128e_3lvl": "spherical blast r=0.1, (1,10)|(0.125,0.1), +-1e-3 rho noise",
           "kh_256e_5lvl": "shear layer rho 2|1, u +-0.5, p 2.5, seeded v modes 1-8",
           "multi_256": "256 seeded blast/Sod instances, 32-128^3, 2-4 levels"}
    eff = max(pb.n0) * 16 << pb.lmax
    return {"workload": name, "instances": len(pbs), "levels": pb.lmax + 1, "effective_grid": eff,
            "block": "16^3 + 4 halo", "ic": ics[name], "eps": pb.eps, "cfl": pb.cfl,
            "path": "batched FP32, steps replayed from a hipGraph, next step queued ahead"}


def counted_traffic(name: str, kernel: str):
    """HBM bytes per launch of the given fused-kernel variant on a workload from the
    committed counter summary, or None when the kernel source changed since."""
    import hashlib
    try:
        prof = json.load(open(os.path.join(ROOT, "profiles", f"rhs_update_{name}_counters.json")))
        src = open(os.path.join(ROOT, prof["source"]), "rb").read()
    except (OSError, KeyError, ValueError):
        return None
    if hashlib.sha256(src).hexdigest()[:16] != prof["source_sha256_16"]:
        return None
    return prof.get("traffic_bytes_per_dispatch", {}).get(kernel)


def kernel_name(shape) -> str:
    """Demangled name of the fused kernel's instantiation for a variant shape."""
    gp, tpb, wpe, ptr = shape
    b = lambda v: "true" if v else "false"
    return f"k_rhs_update<float, {gp}, {abs(tpb)}, {b(tpb < 0)}, {wpe}, 0>"


def flops_per_cell_update(llf_fraction: float) -> float:
    return 3.0 * (17.0 / 16.0) * (FACE_BASE + 5.0 * llf_fraction * LLF_EXTRA) + UPDATE


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_cpu():
    """CPU model, physical cores and logical CPUs this process may run on."""
    model, cores = "unknown", set()
    try:
        phys = core = None
        for line in open("/proc/cpuinfo"):
            k, _, v = line.partition(":")
            k, v = k.strip(), v.strip()
            if k == "model name":
                model = v
            elif k == "physical id":
                phys = v
            elif k == "core id":
                core = v
            elif not k and phys is not None:
                cores.add((phys, core))
                phys = core = None
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = os.cpu_count() or 1
    return model, len(cores) or None, allowed


def leafset(g, inst=0):
    return frozenset(tuple(int(v) for v in r[2:6]) for r in g.blocks() if r[6] == 1 and r[1] == inst)


def oracle_leafset(o):
    return frozenset(tuple(int(v) for v in r[:4]) for r in o.blocks() if r[4] == 1)


def l1(o, g, q):
    """Volume-weighted L1 difference of component q over the leaves both trees share."""
    import numpy as np
    so, sg = o.leaf_states(), g.leaf_states()
    return sum(np.abs(sg[k][q] - v[q]).sum() * o.problem.dx(k[0]) ** 3 for k, v in so.items() if k in sg)


def parity_leg(name, pbs, g, steps, want_cpu):
    """The oracle and the GPU solver g (freshly initialised) run `steps` steps from the same
    initial condition.  Returns the parity summary, the oracle's rate and LLF fraction."""
    from oracle import oracle
    pb = pbs[0]
    t0 = time.perf_counter()
    o = oracle.Sim(pb).init()
    log(f"[bench] oracle algo:Init of {name}: {time.perf_counter() - t0:.1f} s, "
        f"{len(o.blocks())} blocks")
    same = [oracle_leafset(o) == leafset(g)]
    cells, secs, llf = 0, 0.0, []
    for s in range(steps):
        leaves = int((o.blocks()[:, 4] == 1).sum())
        t0 = time.perf_counter()
        o.step()
        secs += time.perf_counter() - t0
        cells += 3 * leaves * 16 ** 3
        llf.append(o.llf_fraction)
        g.step()
        same.append(oracle_leafset(o) == leafset(g))
        log(f"[bench] parity step {s}: oracle {secs:.1f} s so far, trees identical {same[-1]}")
    g.check()
    e_rho, e_E = l1(o, g, 0), l1(o, g, 4)
    vol = float(pb.n0[0] * pb.n0[1] * pb.n0[2]) * (16 * pb.dx0) ** 3
    par = {"steps": steps, "trees_identical": f"{sum(same)}/{len(same)} (init + steps)",
           "l1_rho": e_rho, "l1_E": e_E, "domain_volume": vol,
           "l1_over_common_leaves_only": not all(same)}
    cpu = None
    if want_cpu:
        model, phys, allowed = host_cpu()
        cpu = {"value": cells / secs, "unit": "cell-updates/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"steps 1-{steps} of {name} after the oracle's own algo:Init "
                         f"({cells / 3 / steps / 4096:.0f} leaves; FP64, OpenMP over blocks)",
               "physical_cores": phys, "logical_cpus_allowed": allowed, "cpu_model": model}
    return par, cpu, sum(llf) / len(llf)


def run_gpu(pbs, dtype, batched, warmup, steps, timing=False, variant=None, prepare=None):
    """Init, `warmup` steps (the first ones through `prepare(g)` if given), autotune the
    fused kernel's launch shape (batched FP32; or take `variant`), then `steps` timed
    steps through the library's step loop (mrfv_run)."""
    import torch
    from paper_2012_04385_amd.mrfv import Solver
    t0 = time.perf_counter()
    g = Solver(pbs, dtype=dtype, batched=batched, capacity=capacity_for(pbs)).init()
    log(f"[bench] {dtype} batched={batched}: algo:Init {time.perf_counter() - t0:.1f} s, "
        f"{g.stats()[1]} leaves")
    done = prepare(g) if prepare else 0
    for _ in range(max(warmup - done, 0)):
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
    cells = 3 * g.run(steps)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    g.check()
    kt = g.kernel_time() if timing else None
    return g, cells, secs, kt


def capacity_for(pbs):
    """Slots for the benchmark contexts: every instance fully refined, at most 60,000 (a
    localised feature on a deep tree never comes near its full refinement)."""
    from paper_2012_04385_amd.mrfv import slot_capacity_for
    return min(slot_capacity_for(pbs), 60000)


def lts_leg(pbs, dtype, warmup, macro_steps):
    """Local time stepping (mrfv_step_lts on a per-block context in `dtype`: FP32 takes the
    flux divergence from the fused stage kernel in its default launch shape, FP64 from the
    plain flux kernel) against global steps of the same context from the same start, and
    in FP32 against global steps of the batched path in the same shape (mrfv_run): simulated time
    advanced per second of wall clock (time to solution), and cell-updates per second per
    RK stage (leaf cells times their own steps)."""
    import torch
    from paper_2012_04385_amd.mrfv import Solver
    lmax = pbs[0].lmax
    path = ("fused stage kernel (flux divergence) + local time stepping kernels" if dtype == "f32"
            else "plain per-block kernels")
    out = {"dtype": dtype, "path": path, "macro_steps": macro_steps,
           "micro_steps_per_macro_step": 1 << lmax}
    g = Solver(pbs, dtype=dtype, batched=0, capacity=capacity_for(pbs)).init()
    if dtype == "f32":
        out["launch_shape"] = g.rhs_variants()[g.set_rhs_variant(-1)]
    for _ in range(warmup):
        g.step_lts()
    g.check()
    torch.cuda.synchronize()
    sim, cells = 0.0, 0
    t0 = time.perf_counter()
    for _ in range(macro_steps):
        cells += 3 * g.step_lts()
        sim += float(g.dt.cpu()[0]) * (1 << lmax)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    g.check()
    out.update({"ms_per_macro_step": 1e3 * secs / macro_steps, "sim_time_per_s": sim / secs,
                "cell_updates_per_s": cells / secs, "leaves_final": g.stats()[1]})
    free(g)
    g = Solver(pbs, dtype=dtype, batched=0, capacity=capacity_for(pbs)).init()
    for _ in range(warmup * (1 << lmax)):
        g.step()
    g.check()
    torch.cuda.synchronize()
    sim_g, steps = 0.0, 0
    t0 = time.perf_counter()
    while sim_g < sim:
        g.step()
        sim_g += float(g.dt.cpu()[0])
        steps += 1
    torch.cuda.synchronize()
    secs_g = time.perf_counter() - t0
    g.check()
    free(g)
    out.update({"global_steps": steps, "global_ms_per_step": 1e3 * secs_g / steps,
                "global_sim_time_per_s": sim_g / secs_g,
                "time_to_solution_speedup": (sim / secs) / (sim_g / secs_g)})
    if dtype == "f32":
        # global steps on the fused batched path in the launch shape the local time
        # stepping context used, as a user runs them (mrfv_run: step graphs, the next step
        # queued ahead): as many steps as the plain global leg took, whose CFL steps these
        # repeat up to FP32 rounding, so they cover the same simulated time
        g = Solver(pbs, dtype=dtype, batched=2, capacity=capacity_for(pbs)).init()
        g.run(warmup * (1 << lmax))
        g.check()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.run(steps)
        torch.cuda.synchronize()
        secs_f = time.perf_counter() - t0
        g.check()
        free(g)
        out.update({"fused_global_ms_per_step": 1e3 * secs_f / steps,
                    "speedup_vs_fused_global": (sim / secs) / (sim_g / secs_f)})
    # the path's own roofline: the stiffened-gas FLOP model per cell-update over the whole
    # macro step's rate (a lower bound of its flux kernel's rate)
    peak = PEAK_FP32_VECTOR if dtype == "f32" else PEAK_FP64_VECTOR
    fpc = flops_per_cell_update(0.5)
    out["roofline"] = {"bound": "alu", "achieved": out["cell_updates_per_s"] * fpc / 1e12,
                       "peak": peak / 1e12, "unit": "TFLOP/s", "frac": out["cell_updates_per_s"] * fpc / peak,
                       "basis": "whole-macro-step rate x FLOP model (LLF fraction 0.5 assumed)"}
    out["cpu_baseline"] = lts_oracle_sample()
    return out


def lts_oracle_sample():
    """The oracle's local time stepping timed on a bounded sample: one macro step of a
    four-level periodic tree (levels 0-3, one- and two-level jumps, a Gaussian pulse)."""
    import numpy as np
    from oracle import oracle
    from paper_2012_04385_amd import workloads as W
    pb = W.uniform_flow(lmax=3, n0=(2, 2, 2))
    sim = oracle.Sim(pb, adapt=0).init()
    for args in [(1, 1, 1, 1), (1, 2, 1, 1), (2, 3, 2, 2), (1, 0, 3, 0)]:
        sim.refine(*args)
    sim.coarsen(0, 1, 0, 1)
    for n, r in enumerate(sim.blocks()):
        lvl, bx, by, bz = (int(v) for v in r[:4])
        h = pb.dx(lvl)
        ar = np.arange(16) + 0.5
        z, y, x = np.meshgrid((bz * 16 + ar) * h, (by * 16 + ar) * h, (bx * 16 + ar) * h, indexing="ij")
        g = np.exp(-((x - 0.45) ** 2 + (y - 0.5) ** 2 + (z - 0.55) ** 2) / 0.01)
        rho, p = 1.0 + 0.5 * g, 1.0 + 2.0 * g
        blk = sim.get_block(n)
        blk[:, 4:20, 4:20, 4:20] = np.stack([rho, 0.4 * rho, -0.2 * rho, 0.3 * rho,
                                            p / 0.4 + 0.5 * rho * 0.29])
        sim.set_block(n, blk)
    sim.project()
    cells = 3 * sum((1 << int(r[0])) * 16 ** 3 for r in sim.blocks() if r[4] == 1)
    t0 = time.perf_counter()
    sim.step_lts()
    secs = time.perf_counter() - t0
    model, phys, allowed = host_cpu()
    return {"value": cells / secs, "unit": "cell-updates/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "one LTS macro step of a 4-level periodic test tree (FP64, OpenMP over blocks)",
            "physical_cores": phys, "logical_cpus_allowed": allowed, "cpu_model": model}


def eos_leg(warmup, steps):
    """The Sod tube of Sec. "Influence of Equation of State" (l_max 3) with Tait's equation
    and with the stiffened gas, plain kernels, FP32 and FP64: cell-updates per second and
    their ratio (Tait evolves four of the five components)."""
    from paper_2012_04385_amd import workloads as W
    out = {"workload": "sod tube, 256 cells effective along x, l_max 3", "path": "plain per-block kernels",
           "steps": steps, "warmup": warmup}
    for dtype in ("f32", "f64"):
        for eos in ("stiffened", "tait"):
            pbs = [W.sod_tait_mr3(eos=eos, steps=warmup + steps)]
            g, cells, secs, _ = run_gpu(pbs, dtype, 0, warmup, steps)
            out[f"{eos}_{dtype}"] = {"cell_updates_per_s": cells / secs, "ms_per_step": 1e3 * secs / steps,
                                     "leaves_final": g.stats()[1]}
            free(g)
            log(f"[bench] {eos} {dtype}: {cells / secs:.4e} cell-updates/s")
        out[f"tait_time_per_cell_update_vs_stiffened_{dtype}"] = (
            out[f"stiffened_{dtype}"]["cell_updates_per_s"] / out[f"tait_{dtype}"]["cell_updates_per_s"])
    # the oracle on the same tube with Tait's equation: five steps after its algo:Init
    from oracle import oracle
    pb = W.sod_tait_mr3(eos="tait", steps=5)
    sim = oracle.Sim(pb).init()
    cells = 0
    t0 = time.perf_counter()
    for _ in range(5):
        cells += 3 * 16 ** 3 * int((sim.blocks()[:, 4] == 1).sum())
        sim.step()
    secs = time.perf_counter() - t0
    model, phys, allowed = host_cpu()
    out["cpu_baseline_tait"] = {"value": cells / secs, "unit": "cell-updates/s", "cores": oracle.num_threads(),
                                "kind": "oracle", "sample": "steps 1-5 of the tube with Tait's equation (FP64)",
                                "physical_cores": phys, "logical_cpus_allowed": allowed, "cpu_model": model}
    return out


def rti_leg(ks, t_end, dtype="f64"):
    """The Rayleigh-Taylor growth-rate study (Sec. "Rayleigh-Taylor instability") at the
    settings of its table of inputs for Atwood number 0.5 (l_max 3, 128 cells per
    wavelength, 1:10 domain, amplitude 0.05 / k), viscous plain kernels: per wavenumber the
    growth rate n = d/dt ln(d / d0), fitted over 3 / sqrt(k) <= t <= t_end / sqrt(k) (past the
    start-up transient, before the amplitude leaves the linear regime), against the root of
    eq:SinglePhaseGrowth, and the solver's rate in cell-updates per second."""
    import math
    from oracle import oracle
    from paper_2012_04385_amd import rti
    from paper_2012_04385_amd import workloads as W
    from paper_2012_04385_amd.mrfv import Solver
    rh, rl, mu = W.RTI_FLUIDS[0.5]
    out = {"workload": "Rayleigh-Taylor, At 0.5, rho 1.5 | 0.5, mu 0.1, g 1, l_max 3, 128 cells per "
                       "wavelength, 1280 along y", "dtype": dtype, "path": "plain per-block kernels + viscous",
           "fit": "least-squares slope of ln d(t) over 3/sqrt(k) <= t <= t_end/sqrt(k)", "runs": []}
    for k in ks:
        pb = W.rti(k=k, atwood=0.5, lmax=3)
        n_th = oracle.rti_growth_rate(k, rh, rl, mu, 1.0)
        scale = 1.0 / math.sqrt(k)   # time scale of the instability ~ 1 / sqrt(At g k)
        g = Solver([pb], dtype=dtype, batched=False).init()
        ts, ds = [0.0], [rti.displacement(g, pb)]
        cells, steps = 0, 0
        t0 = time.perf_counter()
        while g.time[0] < t_end * scale:
            for _ in range(25):
                cells += 3 * g.leaf_cells()
                g.advance(1)
            steps += 25
            ts.append(float(g.time[0]))
            ds.append(rti.displacement(g, pb))
            if steps % 2500 == 0:
                log(f"[bench] rti k={k}: step {steps}, t {ts[-1]:.3f}, d/d0 {ds[-1] / ds[0]:.3f}")
        secs = time.perf_counter() - t0
        try:
            n = rti.growth_rate(ts, ds, 3.0 * scale, t_end * scale)
        except ValueError:   # a run shorter than the fit window (profiling): no rate
            n = float("nan")
        run = {"k": k, "n": n, "n_eq_single_phase_growth": n_th, "ratio": n / n_th,
               "n_inviscid": math.sqrt(0.5 * k), "steps": steps, "t_end": ts[-1],
               "amplitude_growth": ds[-1] / ds[0], "leaves_final": g.stats()[1],
               "cell_updates_per_s": cells / secs, "wall_s": secs}
        out["runs"].append(run)
        log(f"[bench] rti k={k}: n {n:.4f} vs {n_th:.4f} ({n / n_th:.3f}), {cells / secs:.3e} cell-updates/s")
        free(g)
    return out


def schemes_leg(warmup, steps, parity_steps=2):
    """The four flux kernels of Sec. "Numerical Scheme" on the weak-scaling case of Sec. "Weak
    Scaling" in its one-core size (Woodward-Colella blast along y, l_max 3, 128 x 512 x 128,
    CFL 0.9): per kernel the FP32 batched path's rate (step graph, autotuned shape) after
    `parity_steps` steps run next to the oracle (identical trees, L1 differences), and the
    FP64 plain path's rate; times relative to the standard configuration (Roe-WENO5)."""
    from paper_2012_04385_amd import workloads as W
    out = {"workload": "Woodward-Colella blast along y, 128 x 512 x 128 effective, l_max 3, CFL 0.9",
           "steps": steps, "warmup": warmup, "kernels": {}}
    for scheme in ("roe_weno5", "roe_teno5", "llf_weno5", "hllc_wao53"):
        pbs = [W.wc_blast_mr4(scheme, steps=warmup + steps)]
        res = {}

        def prepare(g):
            res["parity"], _, res["llf"] = parity_leg(pbs[0].name, pbs, g, parity_steps, False)
            return parity_steps

        from paper_2012_04385_amd.mrfv import MrfvError
        r = {}
        for cfl in (0.9, 0.5):
            # a kernel that stops with a non-physical state at the paper's CFL 0.9 is reported
            # and measured at CFL 0.5
            pbs = [W.wc_blast_mr4(scheme, steps=warmup + steps)]
            pbs[0].cfl = cfl
            try:
                g, cells, secs, _ = run_gpu(pbs, "f32", 2, warmup, steps, prepare=prepare)
            except MrfvError as e:
                r[f"fp32_error_cfl_{cfl}"] = str(e)
                import torch
                torch.cuda.empty_cache()
                continue
            r.update({"cell_updates_per_s": cells / secs, "ms_per_step": 1e3 * secs / steps, "fp32_cfl": cfl,
                      "leaves_final": g.stats()[1], "parity_vs_oracle": res["parity"],
                      "autotuned_shape": g.rhs_variants()[g.tuned["choice"]]})
            free(g)
            break
        pbs = [W.wc_blast_mr4(scheme, steps=warmup + steps)]
        g, c64, s64, _ = run_gpu(pbs, "f64", 0, warmup, steps)
        free(g)
        r["fp64_plain_cell_updates_per_s"] = c64 / s64
        out["kernels"][scheme] = r
        log(f"[bench] {scheme}: {r.get('cell_updates_per_s', float('nan')):.3e} cell-updates/s FP32 batched "
            f"(CFL {r.get('fp32_cfl')}), {r['fp64_plain_cell_updates_per_s']:.3e} FP64 plain, "
            f"parity {r.get('parity_vs_oracle', {}).get('trees_identical')} "
            f"L1(rho) {r.get('parity_vs_oracle', {}).get('l1_rho', float('nan')):.1e}")
    ref = out["kernels"]["roe_weno5"]
    for k, r in out["kernels"].items():
        # time per cell-update relative to the standard configuration
        if "cell_updates_per_s" in r and "cell_updates_per_s" in ref:
            r["time_vs_standard_fp32"] = ref["cell_updates_per_s"] / r["cell_updates_per_s"]
        r["time_vs_standard_fp64"] = ref["fp64_plain_cell_updates_per_s"] / r["fp64_plain_cell_updates_per_s"]
    return out


def free(g):
    import torch
    g.close()
    del g
    torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="shockblobs_512e_6lvl", choices=WORKLOADS)
    ap.add_argument("--parity-steps", type=int, default=2,
                    help="first steps also run by the oracle (parity and CPU baseline)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle (parity, CPU baseline)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 plain path")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the extra keys (config 2, local time stepping, Tait's equation)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a device copy of 512 MiB (calibrates HBM byte counters)")
    ap.add_argument("--lts", action="store_true",
                    help="only run local time stepping against global steps (per-block context; FP32 takes "
                         "the flux divergence from the fused kernel)")
    ap.add_argument("--lts-macro-steps", type=int, default=2)
    ap.add_argument("--eos-compare", action="store_true",
                    help="only run the Sod tube with Tait's equation against the stiffened gas "
                         "(plain kernels)")
    ap.add_argument("--schemes", action="store_true",
                    help="only run the four flux kernels on the weak-scaling blast (Sec. \"Weak Scaling\")")
    ap.add_argument("--rti", action="store_true",
                    help="only run the Rayleigh-Taylor growth-rate study (viscous plain kernels)")
    ap.add_argument("--rti-k", default="1", help="comma-separated wavenumbers of --rti")
    ap.add_argument("--rti-t-end", type=float, default=4.5,
                    help="end of the run and of the fit window, in units of 1/sqrt(k)")
    ap.add_argument("--proposer-gain", action="store_true",
                    help="only run the learned-proposer gain test (6-level shock-blobs workload)")
    args = ap.parse_args()
    if args.proposer_gain:
        from paper_2012_04385_amd.proposer import gain_test
        print(json.dumps(gain_test(log=log)), flush=True)
        return
    if args.lts:
        for dtype in ("f32", "f64"):
            r = lts_leg(problems(args.workload, 10 ** 6), dtype, 1, args.lts_macro_steps)
            log(f"[bench] LTS {dtype}: {r['ms_per_macro_step']:.1f} ms per macro step, "
                f"time-to-solution speed-up {r['time_to_solution_speedup']:.2f}")
            print(json.dumps(dict(r, workload=args.workload)), flush=True)
        return
    if args.schemes:
        print(json.dumps(schemes_leg(3, 22)), flush=True)
        return
    if args.rti:
        ks = [float(v) for v in args.rti_k.split(",")]
        print(json.dumps(rti_leg(ks, args.rti_t_end)), flush=True)
        return
    if args.eos_compare:
        print(json.dumps(eos_leg(args.warmup, args.steps)), flush=True)
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
              "(the library runs on one GPU; how the path would shard across GPUs is described, "
              "not implemented)", file=sys.stderr)
        sys.exit(2)

    name = args.workload
    nsteps = args.warmup + args.steps
    pbs = problems(name, nsteps)
    log(f"[bench] workload {name}: FP32 batched, warmup {args.warmup}, timed {args.steps}")
    oracle_leg = not args.no_cpu and len(pbs) == 1
    res = {}

    def prepare(g):
        if not oracle_leg:
            return 0
        res["parity"], res["cpu"], res["llf"] = parity_leg(name, pbs, g, args.parity_steps, True)
        return args.parity_steps

    g32, cells, secs, _ = run_gpu(pbs, "f32", 2, args.warmup, args.steps, prepare=prepare)
    value = cells / secs
    tuned = g32.tuned
    full = sum(pb.n0[0] * pb.n0[1] * pb.n0[2] * 8 ** pb.lmax * 16 ** 3 for pb in pbs)
    stats = {"leaves_final": g32.stats()[1], "compression": g32.stats()[2] / full,
             "host_adaptation_ms_per_step": {k: v / max(g32.step_timing()["steps"], 1)
                                             for k, v in g32.step_timing().items() if k != "steps"}}
    log(f"[bench] FP32 batched, step graph: {value:.4e} cell-updates/s, "
        f"{1e3 * secs / args.steps:.3f} ms/step")
    free(g32)
    # same steps with eager launches and HIP events around every fused-kernel launch
    ge, cells_e, secs_e, kt = run_gpu(pbs, "f32", 1, args.warmup, args.steps, timing=True,
                                      variant=tuned["choice"])
    value_eager = cells_e / secs_e
    log(f"[bench] FP32 batched, eager + kernel events: {value_eager:.4e} cell-updates/s")
    free(ge)

    extra = {}
    if not args.no_fp64:
        g64, cells64, secs64, _ = run_gpu(pbs, "f64", 0, args.warmup, args.steps)
        free(g64)
        v64 = cells64 / secs64
        log(f"[bench] FP64 plain: {v64:.4e} cell-updates/s")
        extra.update({"fp64_plain_value": v64, "speedup_vs_fp64_plain": value / v64})
        # the baseline's own roofline: the same FLOP model per cell-update over the whole
        # step's rate (an upper bound on the plain path's flux kernel rate) against FP64 peak
        fpc64 = flops_per_cell_update(res.get("llf", 0.5))
        extra["fp64_plain_roofline"] = {"bound": "alu", "achieved": v64 * fpc64 / 1e12,
                                        "peak": PEAK_FP64_VECTOR / 1e12, "unit": "TFLOP/s",
                                        "frac": v64 * fpc64 / PEAK_FP64_VECTOR,
                                        "basis": "whole-step rate x FLOP model"}

    if not args.no_extra and name != "blast_128e_3lvl":
        pb2 = problems("blast_128e_3lvl", 50)
        gb, cb, sb, _ = run_gpu(pb2, "f32", 2, 5, 45)
        free(gb)
        c2 = {"value": cb / sb, "ms_per_step": 1e3 * sb / 45, "steps": 45, "warmup": 5}
        if not args.no_fp64:
            gb, cb64, sb64, _ = run_gpu(pb2, "f64", 0, 5, 45)
            free(gb)
            c2["fp64_plain_value"] = cb64 / sb64
            c2["speedup_vs_fp64_plain"] = c2["value"] / c2["fp64_plain_value"]
        extra["blast_128e_3lvl"] = c2
        log(f"[bench] config 2 (blast_128e_3lvl): {c2['value']:.4e} cell-updates/s")

    if not args.no_extra:
        try:
            lt = lts_leg(pbs, "f32", 1, 2)
            extra["local_time_stepping"] = lt
            log(f"[bench] LTS f32: time-to-solution speed-up {lt['time_to_solution_speedup']:.2f}")
        except Exception as e:   # reported, not fatal: the headline stands on its own
            extra["local_time_stepping"] = {"error": str(e)}
        extra["tait_vs_stiffened"] = eos_leg(5, 30)

    launches, total_ms, kcells = kt
    avg_s = total_ms / 1e3 / max(launches, 1)
    cells_per_launch = kcells / max(launches, 1)
    llf = res.get("llf", 0.5)
    fpc = flops_per_cell_update(llf)
    achieved = cells_per_launch * fpc / avg_s
    kname = kernel_name(tuned["shapes"][tuned["choice"]])
    hbm = cells_per_launch * BYTES_PER_CELL_UPDATE / avg_s
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VECTOR / 1e12,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR,
            "traffic": counted_traffic(name, kname),
            "kernel": kname, "avg_launch_ms": avg_s * 1e3, "launches": launches,
            "cells_per_launch": cells_per_launch, "flop_per_cell_update": fpc,
            "llf_fraction": llf, "llf_source": "oracle, parity steps" if "llf" in res else "assumed",
            "peak_unpacked_fp32": PEAK_FP32_UNPACKED / 1e12,
            "frac_of_unpacked": achieved / PEAK_FP32_UNPACKED,
            "algorithmic_hbm_gbs": hbm / 1e9, "algorithmic_hbm_frac": hbm / PEAK_HBM,
            "bytes_per_cell_update": BYTES_PER_CELL_UPDATE}
    out = {"metric": "cell-updates/s per RK stage (FP32 batched MR RK3)", "value": value,
           "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * secs / args.steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": dict(describe(name, pbs), **{k: stats[k] for k in ("leaves_final", "compression")}),
           "roofline": roof, "cpu_baseline": res.get("cpu")}
    if "parity" in res:
        out["parity_vs_oracle"] = res["parity"]
    out["value_eager_launches"] = value_eager
    out["autotune"] = tuned
    out["host_adaptation_ms_per_step"] = stats["host_adaptation_ms_per_step"]
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

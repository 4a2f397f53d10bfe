"""Training and evaluation of the learned refinement proposer.

The proposer is not part of the paper's method.  A 192-64-64-3 network reads, for every
leaf at the start of a step, 4^3 sub-cube means of (rho, |grad rho|, p) and predicts the
flag the Harten detail threshold will give that leaf at the end of the step (refine /
keep / coarsen).  The solver commits the proposed flags on the host tree, builds and
uploads the resulting tables while the device integrates, and adopts them only when the
judged flags are identical; the committed flags are always the judge's, so the solution
does not depend on the proposer.

Labels come from the solver's own judged flags (mrfv_last_flags) on the 3-level blast and
the 5-level Kelvin-Helmholtz workloads, and on shock-blobs runs with other seeds than the
evaluated one: within their step counts the first two only ever keep (their trees settle
during initialisation), so without the latter no refine or coarsen label would exist.
The single-level Sod workload has no flags and is not used.  Training (forward, backward,
Adam) runs on the GPU.

`gain_test` runs the 6-level shock-blobs workload three times -- proposer off, persistence
(the proposal is "no change") and the trained network -- and reports step time, the host
time of the adaptation phase, precision and recall per class, hits, and staged tables that
were not adopted; the final states must be bitwise identical.
"""
import hashlib
import time

import numpy as np

from . import workloads as W
from .mrfv import MLP, Solver, collect_training_data, proposer_stats, set_proposer


def training_sources(blast_steps: int = 50, kh_steps: int = 20, blob_steps: int = 100,
                     blob_seeds=(11, 12)):
    """(name, problem, steps) of the label sources."""
    src = [("blast_128e_3lvl", W.blast_mr3(steps=blast_steps), blast_steps),
           ("kh_256e_5lvl", W.kh_mr5(steps=kh_steps), kh_steps)]
    for k in blob_seeds:
        src.append((f"shockblobs_seed{k}", W.shock_blobs_mr6(seed_k=k, steps=blob_steps), blob_steps))
    return src


def collect(sources):
    """Features and judged classes of every leaf of every step of the sources, and a step
    id per row (unique over the sources; the first step of each source has the lowest id
    of that source)."""
    import torch
    Xs, ys, ks, info = [], [], [], {}
    base = 0
    for name, pb, steps in sources:
        g = Solver([pb], dtype="f32", batched=2).init()
        X, y, k = collect_training_data(g, steps, with_steps=True)
        Xs.append(X)
        ys.append(y)
        ks.append(k + base)
        base += steps
        info[name] = np.bincount(y, minlength=3).tolist()
        del g
    return torch.cat(Xs), np.concatenate(ys), np.concatenate(ks), info


def gated_steps(y, k, first_ids):
    """Step ids on which the solver runs the network: the first step of a run and every step
    that follows a step whose judge changed the tree."""
    changed = set(np.unique(k[y != 1]).tolist())
    return sorted(set(first_ids) | {s + 1 for s in changed if s + 1 in set(k.tolist()) and s + 1 not in first_ids})


def train(X, y, epochs: int = 30, lr: float = 3e-3, batch: int = 4096, seed: int = 0,
          max_rows: int = 65536):
    """Class-weighted Adam training on the device; returns the network and the loss
    before and after."""
    mlp = MLP(max_rows=max_rows)
    mlp.init_params(seed=seed)
    cnt = np.bincount(y, minlength=3).astype(np.float64)
    w = np.where(cnt > 0, cnt.sum() / np.maximum(cnt, 1) / 3.0, 0.0).astype(np.float32)
    n_eval = min(len(y), batch)
    l0, _ = mlp.loss_grad(X[:n_eval], y[:n_eval], w, want_grad=False)
    mlp.train(X, y, epochs=epochs, lr=lr, batch=batch, seed=seed, class_w=w)
    l1, _ = mlp.loss_grad(X[:n_eval], y[:n_eval], w, want_grad=False)
    return mlp, float(l0), float(l1)


def step_hits(z, y, k, steps, shift):
    """Steps (of `steps`) on which the argmax proposal with the keep logit raised by
    `shift` equals the judge's classes on every leaf."""
    zz = z.copy()
    zz[:, 1] += shift
    wrong = zz.argmax(axis=1) != y
    bad = set(np.unique(k[wrong]).tolist())
    return sum(1 for s in steps if s not in bad)


def calibrate_keep_bias(mlp, X, y, k, steps):
    """Raise the keep logit's bias to the value at which the network's proposal is exact
    on the most of the given training steps (those the solver runs it on): class
    weighting biases the argmax towards the rare classes, and one wrong leaf makes a whole
    step's staged tree useless.  Among equally good values the largest (fewest change
    proposals) is taken.  Returns the bias shift."""
    import torch
    b = min(32768, mlp.max_rows)
    z = torch.cat([mlp.forward(X[a:a + b]) for a in range(0, X.shape[0], b)]).cpu().numpy()
    sel = np.isin(k, steps)
    m = np.maximum(z[sel, 0], z[sel, 2]) - z[sel, 1]   # margin of a change over keep
    cand = np.unique(np.concatenate([[0.0], np.maximum(m, 0.0) + 1e-3]))
    if len(cand) > 512:   # a coarse grid of the margins' quantiles is enough
        cand = np.unique(np.quantile(cand, np.linspace(0.0, 1.0, 512)))
        cand = np.append(cand, m.max() + 1e-3 if len(m) else 0.0)
    best, shift = -1, 0.0
    for c in cand:
        h = step_hits(z, y, k, steps, float(c))
        if h >= best:
            best, shift = h, float(c)
    p = mlp.get_params()
    p[-3 + 1] += shift
    mlp.set_params(p)
    return shift


def leaf_digest(g) -> str:
    """SHA-256 of the leaf interiors in (instance, level, bx, by, bz) order."""
    import torch
    info = g.blocks()
    sel = info[info[:, 6] == 1]
    order = np.lexsort((sel[:, 5], sel[:, 4], sel[:, 3], sel[:, 2], sel[:, 1]))
    slots = torch.as_tensor(sel[order, 0], device=g.device)
    h = hashlib.sha256()
    for a in range(0, len(slots), 1024):
        blk = g.U[slots[a:a + 1024], :, 4:20, 4:20, 4:20].contiguous().cpu().numpy()
        h.update(blk.tobytes())
    return h.hexdigest()


def run_mode(pb, steps: int, mode: int, mlp=None, variant=None):
    import torch
    g = Solver([pb], dtype="f32", batched=2).init()
    if variant is not None:
        g.set_rhs_variant(variant)
    if mode:
        set_proposer(g, mlp, mode)
    torch.cuda.synchronize()
    cells = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        cells += 3 * g.leaf_cells()
        g.step()
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    g.check()
    ht = g.step_timing()
    out = {"ms_per_step": 1e3 * secs / steps, "cell_updates_per_s": cells / secs,
           "host_ms_per_step": {k: ht[k] / max(ht["steps"], 1) for k in ("wait_ms", "commit_ms", "predict_ms")},
           "leaves_final": g.stats()[1]}
    if mode:
        st = proposer_stats(g)
        prf = {}
        for c in ("refine", "keep", "coarsen"):
            tp, fp, fn = st[c]["tp"], st[c]["fp"], st[c]["fn"]
            prf[c] = {"precision": tp / (tp + fp) if tp + fp else None,
                      "recall": tp / (tp + fn) if tp + fn else None, "support": tp + fn}
        out["proposer"] = {"steps": st["steps"], "hits": st["hits"], "network_runs": st["net_runs"],
                           "staged": st["staged"],
                           "adopted": st["adopted"], "wasted_staged": st["staged"] - st["adopted"],
                           "build_ms_per_step": st["build_ms"] / max(st["steps"], 1), "classes": prf}
    out["digest"] = leaf_digest(g)
    return out


def tuned_variant(pb, warm: int = 3) -> int:
    """Launch shape of the fused kernel the autotuner picks on this workload."""
    g = Solver([pb], dtype="f32", batched=2).init()
    for _ in range(warm):
        g.step()
    choice, _ = g.autotune(reps=2)
    del g
    return choice


def gain_test(steps: int = 100, epochs: int = 30, variant=None, log=print):
    import torch
    t0 = time.perf_counter()
    src = training_sources()
    X, y, k, info = collect(src)
    firsts = list(np.cumsum([0] + [s for _, _, s in src[:-1]]))
    gsteps = gated_steps(y, k, firsts)
    log(f"[proposer] {X.shape[0]} labelled leaves, classes (refine, keep, coarsen) by source: {info}; "
        f"{len(gsteps)} steps follow a tree change or start a run")
    mlp, l0, l1 = train(X, y, epochs=epochs)
    log(f"[proposer] trained {epochs} epochs: loss {l0:.4f} -> {l1:.4f} "
        f"({time.perf_counter() - t0:.1f} s with data collection)")
    shift = calibrate_keep_bias(mlp, X, y, k, gsteps)
    pred = np.concatenate([mlp.forward(X[a:a + 32768]).argmax(dim=1).cpu().numpy()
                           for a in range(0, X.shape[0], 32768)])
    train_acc = float((pred == y).mean())
    tr_prec = {}
    for c, name in ((0, "refine"), (2, "coarsen")):
        tp, pp, ap = int(((pred == c) & (y == c)).sum()), int((pred == c).sum()), int((y == c).sum())
        tr_prec[name] = {"precision": tp / pp if pp else None, "recall": tp / ap if ap else None}
    log(f"[proposer] keep bias +{shift:.3f}; training accuracy {train_acc:.5f}, {tr_prec}")
    del X
    torch.cuda.empty_cache()
    pb = W.shock_blobs_mr6(steps=steps)
    if variant is None:
        variant = tuned_variant(pb)
    log(f"[proposer] fused-kernel launch shape {variant} (autotuned) for all modes")
    res = {}
    for name, mode, net in (("off", 0, None), ("persistence", 2, None), ("network", 1, mlp)):
        log(f"[proposer] {pb.name}, {steps} steps, proposer {name}")
        res[name] = run_mode(pb, steps, mode, net, variant)
        log(f"[proposer]   {res[name]['ms_per_step']:.2f} ms/step, host {res[name]['host_ms_per_step']}")
        torch.cuda.empty_cache()
    same = len({r["digest"] for r in res.values()}) == 1
    gain = (res["network"]["ms_per_step"] < res["off"]["ms_per_step"] and
            res["network"]["ms_per_step"] < res["persistence"]["ms_per_step"])
    no_loss = (res["network"]["proposer"]["hits"] >= res["persistence"]["proposer"]["hits"])
    return {"workload": pb.name, "steps": steps, "variant": variant,
            "training": {"sources": info, "loss_before": l0,
            "loss_after": l1, "train_accuracy": train_acc, "epochs": epochs,
            "keep_bias_shift": shift, "train_change_classes": tr_prec,
            "calibration_steps": len(gsteps)},
            "runs": res, "bitwise_identical": same, "network_gain": gain,
            "network_hits_at_least_persistence": no_loss}

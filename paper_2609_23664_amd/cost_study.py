"""Realized-cost logging for the learned cost model.

For a workload (one shared prefix, T tasks with their own suffixes) this
module computes the planner features (host-only, from the library's pass
counts) and realizes the workload on the GPU under both plans: direct per
task (every task from |0...0> through prefix and suffix, with the same cut)
and reuse (prefix once, frozen snapshot, suffixes from it). Workloads with
more than `max_tasks` tasks are realized on their first `max_tasks` tasks
and scaled linearly:
    t_direct(T) = t_direct(k) * T / k,
    t_reuse(T)  = t_prefix + (t_reuse(k) - t_prefix) * T / k.
The execution is the one the planner governs: the default tiered kernels,
after one untimed run of each plan with generated kernels for every pass
structure (compiled, or read from the disk cache, outside the timing), so
every timed pass runs a generated kernel and no compile time enters a label;
then the faster of two timed runs of each plan (alternating) is kept. Each
record carries the fingerprint of the kernel, planner and generator sources
it was measured on (`kernel_fingerprint`). Run as a module to log the
config-5 study:
    python -m paper_2609_23664_amd.cost_study --out costs.jsonl --count 2000
`--precompile` compiles the workloads' generated kernels into the disk
cache without a GPU (hipRTC only), in parallel processes.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time
from typing import Dict, List, Sequence

import numpy as np

N_FEATURES = 12


def feature_vector(n: int, n_tasks: int, prefix_passes: float, suffix_passes: Sequence[float],
                   prefix_gates: float, suffix_gates: float) -> List[float]:
    """The 12 planner features (all scaled to O(1)): qubits, log2 tasks,
    prefix passes, mean/max/min suffix passes, suffix spread, log2 state
    bytes, log analytic direct / reuse bytes, analytic ratio (capped at
    20), prefix fraction of the gates."""
    sp = list(suffix_passes) or [0.0]
    pp = float(prefix_passes)
    sb = 8.0 * (1 << n)
    msp = float(np.mean(sp))
    est_direct = n_tasks * (pp + msp) * 2 * sb
    est_reuse = (pp + n_tasks * msp) * 2 * sb
    return [n / 26.0, math.log2(max(1, n_tasks)) / 8.0, pp / 32.0, msp / 32.0,
            max(sp) / 32.0, min(sp) / 32.0, (max(sp) - min(sp)) / 16.0, math.log2(sb) / 32.0,
            math.log(max(est_direct, 1.0)) / 40.0, math.log(max(est_reuse, 1.0)) / 40.0,
            min(est_direct / max(est_reuse, 1.0), 20.0) / 10.0,
            prefix_gates / max(1.0, prefix_gates + suffix_gates)]


def features(n: int, prefix: Sequence, suffixes: Sequence[Sequence], n_tasks: int,
             tile_bits: int = 14) -> List[float]:
    """Features of a single-prefix workload from the library's pass counts."""
    from .binding import plan_cost
    pp = plan_cost(n, list(prefix), tile_bits)[0] if prefix else 0
    sp = [plan_cost(n, list(s), tile_bits)[0] for s in suffixes] or [0]
    gs = float(np.mean([len(s) for s in suffixes])) if suffixes else 0.0
    return feature_vector(n, n_tasks, pp, sp, len(prefix), gs)


def kernel_fingerprint() -> str:
    """Hash of the library's kernel, planner and generator sources (csrc):
    a realized cost describes the code it was measured on."""
    import hashlib
    import os
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h", ".cpp")):
            h.update(f.encode())
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def realize(ctx, n: int, prefix, suffixes, n_tasks: int) -> Dict[str, float]:
    """Realized ms of direct and reuse execution (scaled to n_tasks)."""
    from . import binding as B
    from .planner import run_workload, plan_workload
    k = len(suffixes)
    tasks = [list(prefix) + list(s) for s in suffixes]
    plan = plan_workload(n, tasks, decide=lambda *a: True)   # cuts at the shared prefix
    # one untimed run of each plan with generated kernels for every pass
    # structure (compiled or loaded now; plans cached, first-touch effects);
    # the timed runs then use the default tiered mode, which finds them
    ctx.set_option(B.QW_OPT_JIT, 2)
    try:
        run_workload(ctx, n, tasks, plan=plan, mode="direct")
        run_workload(ctx, n, tasks, plan=plan, mode="reuse")
    finally:
        ctx.set_option(B.QW_OPT_JIT, 1)
    rds, rrs = [], []
    for _ in range(2):
        rds.append(run_workload(ctx, n, tasks, plan=plan, mode="direct")[2])
        rrs.append(run_workload(ctx, n, tasks, plan=plan, mode="reuse")[2])
    rd = min(rds, key=lambda r: r.realized_ms["total"])
    rr = min(rrs, key=lambda r: r.realized_ms["total"])
    td = rd.realized_ms["total"] * n_tasks / k
    tp = rr.realized_ms.get("prefix", 0.0)
    tr = tp + (rr.realized_ms["total"] - tp) * n_tasks / k
    return {"t_direct_ms": td, "t_reuse_ms": tr, "t_prefix_ms": tp, "tasks_run": k}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--count", type=int, default=2000)
    ap.add_argument("--first", type=int, default=0)
    ap.add_argument("--max-tasks", type=int, default=16)
    ap.add_argument("--last", type=int, default=None, help="stop before this workload index")
    ap.add_argument("--precompile", type=int, default=0,
                    help="compile the generated kernels of the workloads with this many processes "
                         "(no GPU), then exit")
    ap.add_argument("--recheck", type=int, default=0,
                    help="realize this many seeded held-out workloads of the stored labels again at the "
                         "current sources, then compare them with the stored labels and evaluate the MLP "
                         "trained on the stored training split on both")
    args = ap.parse_args(argv)
    if args.recheck:
        return recheck(args.recheck, args.out, args.max_tasks)
    from workloads import gen
    specs = gen.config5_specs(args.count)[args.first:args.last]
    if args.precompile:
        return precompile(specs, args.max_tasks, args.precompile)
    from . import binding as B
    ctx = B.Ctx(0)
    fp = kernel_fingerprint()
    t0 = time.time()
    with open(args.out, "a") as f:
        for i, s in enumerate(specs):
            w = gen.config5_workload(s, max_tasks=args.max_tasks)
            feats = features(w.n, w.prefix, w.suffixes, s.n_tasks)
            r = realize(ctx, w.n, w.prefix, w.suffixes, s.n_tasks)
            rec = {"index": s.index, "n": s.n, "tasks": s.n_tasks, "prefix_layers": s.prefix_layers,
                   "total_layers": s.total_layers, "spread": s.spread, "negative": s.negative,
                   "features": feats, **r, "kernels": "tiered, generated (warm)", "fingerprint": fp}
            f.write(json.dumps(rec) + "\n")
            f.flush()
            if i % 50 == 0:
                print(f"[cost-study] {i + args.first}/{args.count} n={s.n} T={s.n_tasks} "
                      f"direct={r['t_direct_ms']:.2f}ms reuse={r['t_reuse_ms']:.2f}ms "
                      f"elapsed={time.time() - t0:.0f}s", flush=True)
    return 0


def recheck(k: int, out: str, max_tasks: int = 16, procs: int = 12) -> int:
    """Label drift: the realized costs of k held-out workloads (a seeded sample
    of the stored split) taken again at the current sources, written to `out`;
    prints the drift of log(t_direct / t_reuse) against the stored labels and
    the plan regret of the MLP (trained on the stored training split) and of
    the analytic rule on the new and on the stored labels."""
    import multiprocessing as mp
    from workloads import gen
    from . import costmodel as CM
    rows = CM.load_costs()
    train_rows, test_rows = CM.split(rows)
    rng = np.random.default_rng(2026)
    pick = set(int(test_rows[i]["index"]) for i in rng.choice(len(test_rows), size=min(k, len(test_rows)),
                                                               replace=False))
    specs = [s for s in gen.config5_specs(len(rows)) if s.index in pick]
    t0 = time.time()
    seen, items = set(), []
    for s in specs:
        w = gen.config5_workload(s, max_tasks=max_tasks)
        for g in [w.prefix] + list(w.suffixes):
            sig = (w.n, tuple((x[0], tuple(x[1])) for x in g))
            if g and sig not in seen:
                seen.add(sig)
                items.append((w.n, [list(g)]))
    with mp.get_context("spawn").Pool(procs) as pool:
        for i, _ in enumerate(pool.imap_unordered(_precompile_lists, items)):
            if i % 50 == 0:
                print(f"[cost-study] compiled {i}/{len(items)} gate lists, {time.time() - t0:.0f}s", flush=True)
    from . import binding as B
    ctx = B.Ctx(0)
    fp = kernel_fingerprint()
    new = []
    with open(out, "w") as f:
        for i, s in enumerate(specs):
            w = gen.config5_workload(s, max_tasks=max_tasks)
            r = realize(ctx, w.n, w.prefix, w.suffixes, s.n_tasks)
            rec = {"index": s.index, "n": s.n, "tasks": s.n_tasks, "prefix_layers": s.prefix_layers,
                   "total_layers": s.total_layers, "spread": s.spread, "negative": s.negative,
                   "features": features(w.n, w.prefix, w.suffixes, s.n_tasks), **r,
                   "kernels": "tiered, generated (warm)", "fingerprint": fp}
            f.write(json.dumps(rec) + "\n")
            new.append(rec)
            if i % 20 == 0:
                print(f"[cost-study] realized {i}/{len(specs)}, {time.time() - t0:.0f}s", flush=True)
    old = {r["index"]: r for r in rows}
    olds = [old[r["index"]] for r in new]
    drift = np.array([math.log(a["t_direct_ms"] / a["t_reuse_ms"]) - math.log(b["t_direct_ms"] / b["t_reuse_ms"])
                      for a, b in zip(new, olds)])
    model = CM.MLP(ctx, seed=0)
    x, y = CM.arrays(train_rows)
    model.train(x, y, epochs=300)
    model.calibrate(train_rows)
    res = {"count": len(new), "fingerprint": fp, "stored_fingerprints": sorted({b["fingerprint"] for b in olds}),
           "features_equal": bool(all(np.allclose(a["features"], b["features"]) for a, b in zip(new, olds))),
           "log_ratio_drift": {"mean": float(drift.mean()), "abs_median": float(np.median(np.abs(drift))),
                               "abs_p90": float(np.quantile(np.abs(drift), 0.9))},
           "abstain_truth_changed": int(sum((a["t_direct_ms"] <= a["t_reuse_ms"]) != (b["t_direct_ms"] <= b["t_reuse_ms"])
                                            for a, b in zip(new, olds))),
           "new_labels": CM.evaluate(model, new), "stored_labels": CM.evaluate(model, olds)}
    print(json.dumps(res), flush=True)
    return 0


def _precompile_lists(item):
    n, lists = item
    from . import binding as B
    for g in lists:
        B.jit_precompile(n, g, 14)
    return len(lists)


def precompile(specs, max_tasks: int, procs: int) -> int:
    """Compile (hipRTC, no GPU) the generated pass kernels of every distinct
    gate-list structure of `specs` (prefixes and suffixes; the direct path
    cuts at the same boundary, so it runs the same passes) into the disk
    cache, split over `procs` processes."""
    import multiprocessing as mp
    from workloads import gen
    seen, by_n = set(), {}
    for s in specs:
        w = gen.config5_workload(s, max_tasks=max_tasks)
        for g in [w.prefix] + list(w.suffixes):
            sig = (w.n, tuple((x[0], tuple(x[1])) for x in g))
            if g and sig not in seen:
                seen.add(sig)
                by_n.setdefault(w.n, []).append(list(g))
    items = [(n, [g]) for n, gs in sorted(by_n.items()) for g in gs]
    t0 = time.time()
    done = 0
    with mp.get_context("spawn").Pool(procs) as pool:
        for i, c in enumerate(pool.imap_unordered(_precompile_lists, items)):
            done += c
            if i % 100 == 0:
                print(f"[cost-study] compiled {i}/{len(items)} gate lists, {time.time() - t0:.0f}s", flush=True)
    print(f"[cost-study] precompiled {done} gate lists in {time.time() - t0:.0f}s", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

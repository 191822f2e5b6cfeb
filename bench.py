"""Benchmark: VQE tasks/s at 24 qubits, reuse vs direct on one MI355X.

Workload (default): 24 qubits, 8 hardware-efficient layers (RY, RZ on every
qubit, then a CNOT ladder), 6 shared prefix layers, 64 tasks with their own
2-layer suffix, 50 random Pauli strings of weight <= 4 (seeded synthetic
input; no dataset). One step = the whole reuse path: reset the boundary slot,
apply the prefix once, freeze it as the boundary snapshot, replay the 64
suffixes from it and reduce the 64 Pauli-sum expectations to the host.

Prints one JSON line (the contract of this repository's driver).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-direct", action="store_true")
    ap.add_argument("--cpu-tasks", type=int, default=1,
                    help="tasks in the oracle's bounded CPU sample")
    return ap.parse_args()


def main():
    args = _parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2609_23664_amd import binding as B
    from paper_2609_23664_amd.planner import fingerprint
    from workloads import gen

    assert torch.cuda.is_available(), "no GPU"
    w = gen.config2()
    n, T = w.n, w.n_tasks
    terms = w.terms
    prov = fingerprint(n, w.prefix)
    ctx = B.Ctx(0)

    # gate lists marshalled once (host preparation, outside the timed steps;
    # the library's plan cache makes later steps skip planning, which the
    # first, untimed step does)
    prefix = B.GateArray(w.prefix)
    suffixes = [B.GateArray(s) for s in w.suffixes]

    # ---- reuse path: slot 0 = boundary, slots 1..T = tasks
    st = B.State(ctx, n, T + 1)
    slots = list(range(1, T + 1))

    def reuse_step():
        st.reset(0, 1)
        st.apply(0, prefix)
        snap = st.snapshot(0, prov, B.QW_SNAP_FREEZE)
        e = B.run_suffix_batch(ctx, [snap] * T, suffixes, st, slots, terms=terms)
        snap.free()
        return e

    # ---- direct path: every task from |0...0> through prefix then suffix
    dst = None if args.no_direct else B.State(ctx, n, T)
    dslots = list(range(T))

    def direct_step():
        dst.reset(0, T)
        B.run_suffix_batch(ctx, None, [prefix] * T, dst, dslots)
        return B.run_suffix_batch(ctx, None, suffixes, dst, dslots, terms=terms)

    def timed(fn, steps, warmup, profile=False):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        if profile:
            ctx.set_option(B.QW_OPT_PROFILE, 1)
            for k in range(4):
                ctx.kernel_stats(k, reset=True)
        t0 = time.perf_counter()
        out = None
        for _ in range(steps):
            out = fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        stats = None
        if profile:
            stats = [ctx.kernel_stats(k, reset=True) for k in range(4)]
            ctx.set_option(B.QW_OPT_PROFILE, 0)
        return dt, out, stats

    dt_r, e_r, stats = timed(reuse_step, args.steps, args.warmup, profile=True)
    value = T * args.steps / dt_r
    result = {
        "metric": "VQE tasks/s at 24q (reuse, same GPU as direct)",
        "value": round(value, 2),
        "unit": "tasks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt_r / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 (fp32 amplitudes, fp64 accumulation)",
        "data": "synthetic (seeded HEA angles and Pauli terms)",
        "config": {"workload": w.name, "qubits": n, "tasks": T, "prefix_layers": 6,
                   "suffix_layers": 2, "terms": len(terms), "parallelism": "single GPU"},
    }
    if dst is not None:
        dt_d, e_d, _ = timed(direct_step, args.steps, args.warmup)
        result["direct_tasks_per_s"] = round(T * args.steps / dt_d, 2)
        result["speedup_vs_direct"] = round(dt_d / dt_r, 3)
        result["gate_count_prediction"] = round(
            T * (len(w.prefix) + len(w.suffixes[0])) / (len(w.prefix) + T * len(w.suffixes[0])), 3)
        result["reuse_equals_direct"] = bool(e_r == e_d)
    # dominant kernel: gate pass
    n_l, ms, by = stats[0]
    peak = 8000.0
    achieved = by / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    result["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": peak,
                          "unit": "GB/s", "frac": round(achieved / peak, 4), "traffic": None,
                          "kernel": "pass_kernel<14>", "launches": n_l,
                          "avg_launch_ms": round(ms / max(1, n_l), 4)}
    red = stats[1]
    if red[0]:
        result["reducer"] = {"launches": red[0], "avg_launch_ms": round(red[1] / red[0], 4),
                             "GB/s": round(red[2] / (red[1] * 1e-3) / 1e9, 1)}
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_tasks)
    print(json.dumps(result), flush=True)


def cpu_baseline(w, k):
    """The oracle (complex128, OpenMP over amplitudes) on a bounded sample:
    the shared prefix once plus k tasks (suffix + Pauli-sum expectation);
    tasks/s for the full workload is extrapolated as
    T / (t_prefix + T * t_task)."""
    import oracle
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    base = oracle.simulate(w.n, w.prefix)
    t_prefix = time.perf_counter() - t0
    t1 = time.perf_counter()
    for t in range(k):
        psi = oracle.apply_gates(base.copy(), w.n, w.suffixes[t])
        oracle.expect(psi, w.n, w.terms)
    t_task = (time.perf_counter() - t1) / k
    T = w.n_tasks
    return {"value": round(T / (t_prefix + T * t_task), 4), "unit": "tasks/s", "cores": cores,
            "kind": "oracle",
            "sample": f"prefix once ({len(w.prefix)} gates) + {k} task(s) of {T}; "
                      f"t_prefix={t_prefix:.2f}s t_task={t_task:.2f}s"}


if __name__ == "__main__":
    main()

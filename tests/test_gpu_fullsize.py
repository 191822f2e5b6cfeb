"""GPU parity at the full sizes of the prefix-tree workload (20 qubits, 512
leaves, 1,024 shots) and the noisy workload (22 qubits, 256 trajectories,
1,024 shots), in the launch configuration the benchmark times (one recorded
graph per execution): the planned graph's samples equal the direct graph's
bit for bit, and sampled tasks match the oracle (fidelity, and every shot a
valid inverse-CDF pick of the oracle's distribution, at least 99 % of them
identical to the oracle's own draws). Every case prints its name first."""
import sys

import numpy as np
import pytest

import oracle
from workloads import gen

pytestmark = pytest.mark.gpu

FID_TOL = 1e-6
NORM_TOL = 1e-5   # |<psi|psi> - 1|; the derivation is in test_gpu_parity.py


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2609_23664_amd import binding
    assert torch.cuda.is_available()
    c = binding.Ctx(0)
    yield c
    c.sync()


def _check_against_oracle(n, tasks, samples, states, picks, seed, shots, refs=None):
    same = 0
    worst = [0.0, 0.0]
    for k in picks:
        ref = oracle.simulate(n, tasks[k]) if refs is None else refs(k)
        g = states[k].astype(np.complex128)
        inf = 1 - oracle.fidelity(g, ref)
        drift = abs(float(np.vdot(g, g).real) - 1.0)
        worst = [max(worst[0], inf), max(worst[1], drift)]
        assert inf <= FID_TOL, k
        assert drift <= NORM_TOL, k
        cdf = np.cumsum(np.abs(ref) ** 2)
        o = oracle.sample(ref, n, seed, k, shots)
        same += int(np.sum(o == samples[k]))
        assert np.all(np.abs(ref[samples[k]]) > 0), k
        for s_, i in enumerate(samples[k]):
            u = oracle.uniform(seed, k, s_) * cdf[-1]
            lo = cdf[i - 1] if i > 0 else 0.0
            assert lo - 1e-6 <= u <= cdf[i] + 1e-6, (k, s_)
    say(f"  {len(picks)} tasks: worst 1-F={worst[0]:.2e} drift={worst[1]:.2e} "
        f"identical shots {same / (len(picks) * shots):.5f}")
    assert same >= 0.99 * len(picks) * shots


def _run_graphs(ctx, n, tasks, shots, seed, picks):
    from paper_2609_23664_amd import planner as P
    plan = P.plan_workload(n, tasks)
    assert plan.decision == "REUSE"
    out = {}
    for mode in ("plan", "direct"):
        rw = P.record_workload(ctx, n, tasks, plan, shots=shots, seed=seed, mode=mode)
        try:
            rw.replay()
            res = rw.results()
            states = {k: rw.state_host(k) for k in picks}
        finally:
            rw.free()
        out[mode] = (res.samples, states)
    return out


def test_config3_full_size_graph(ctx):
    say("config3 full size: 20q, 512 leaves, 1024 shots, graphs")
    w = gen.config3()
    tasks = [w.leaf_path(k) for k in range(len(w.leaves))]
    # 32 seeded leaves (the first and last among them), every suffix length
    picks = sorted({0, len(tasks) - 1} | set(
        np.random.default_rng(3031).choice(len(tasks), 30, replace=False).tolist()))
    out = _run_graphs(ctx, w.n, tasks, w.shots, w.seed, picks)
    (sp, stp), (sd, std) = out["plan"], out["direct"]
    assert sp.shape == (512, 1024)
    assert np.array_equal(sp, sd)
    for k in picks:
        assert np.array_equal(stp[k], std[k]), k
    _check_against_oracle(w.n, tasks, sp, stp, picks, w.seed, w.shots)


def test_config4_full_size_graph(ctx):
    say("config4 full size: 22q, 256 trajectories, 1024 shots, graphs")
    w = gen.config4()
    tasks = [list(w.prefix) + list(t) for t in w.trajectories]
    jumped = [t for t in range(len(tasks)) if list(w.trajectories[t]) != list(w.suffix)]
    clean = [t for t in range(len(tasks)) if list(w.trajectories[t]) == list(w.suffix)]
    # every trajectory with a jump, and 16 seeded jump-free ones
    picks = sorted(jumped + np.random.default_rng(4041).choice(clean, 16, replace=False).tolist())
    say(f"  {len(jumped)} trajectories with jumps, {len(picks)} checked")
    out = _run_graphs(ctx, w.n, tasks, w.shots, w.seed, picks)
    (sp, stp), (sd, std) = out["plan"], out["direct"]
    assert sp.shape == (256, 1024)
    assert np.array_equal(sp, sd)
    for k in picks:
        assert np.array_equal(stp[k], std[k]), k
    base = oracle.simulate(w.n, w.prefix)   # the oracle's own reuse: bitwise its direct run
    _check_against_oracle(w.n, tasks, sp, stp, picks, w.seed, w.shots,
                          refs=lambda k: oracle.apply_gates(base.copy(), w.n, list(w.trajectories[k])))

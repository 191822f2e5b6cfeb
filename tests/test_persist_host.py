"""Host checks of the persistent launch's claim schedule (qw_persist_schedule,
the function the executor uses): segments tile the claims and descriptors
contiguously, every (task, pass) is swept once in whole units, every
descriptor waits for its task's previous pass or its parent task's last
pass, and every dependency's claims all come before the claims that wait
for it. A simulation of workgroups that take claims in order, decoded as
the kernel decodes them, and hold a claim while its dependency is unmet,
drains every schedule for any number of workgroups (one included), which is
the launch's progress argument."""
import heapq

import numpy as np
import pytest

from paper_2609_23664_amd import binding as B


def _random_tree(rng, n_tasks, max_passes=5, n_kinds=6):
    parents, passes, kinds, units = [], [], [], []
    for t in range(n_tasks):
        parents.append(int(rng.integers(-1, t)) if t and rng.random() < 0.8 else -1)
        p = int(rng.integers(1, max_passes + 1))
        passes.append(p)
        for _ in range(p):
            k = int(rng.integers(n_kinds))
            kinds.append(k)
            units.append(4 if k % 3 == 0 else 16)   # an epilogue structure sweeps rows
    return parents, passes, kinds, units


def _claim_desc(segs, c):
    """The kernel's decoding of claim c: (descriptor, first unit, units)."""
    lo, hi = 0, len(segs)
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if segs[mid][0] <= c:
            lo = mid
        else:
            hi = mid
    claim0, n_claims, desc0, n_descs, chunk, kind, tmaj, units = segs[lo]
    lc = c - claim0
    per = units // chunk
    dl, ul = (lc // per, lc % per) if tmaj else (lc % n_descs, lc // n_descs)
    return desc0 + dl, ul * chunk, chunk


def _check_structure(sch, parents, passes, kinds, units, chunk_max, grid):
    segs, deps, descs = sch["segments"], sch["deps"], sch["descs"]
    base = np.cumsum([0] + list(passes))
    # every (task, pass) exactly once
    assert sorted(map(tuple, descs)) == [(t, k) for t in range(len(passes)) for k in range(passes[t])]
    pos = {tuple(d): i for i, d in enumerate(descs)}
    claim = desc = 0
    for claim0, n_claims, desc0, n_descs, chunk, kind, tmaj, u in segs:
        assert claim0 == claim and desc0 == desc
        assert chunk & (chunk - 1) == 0 and 1 <= chunk <= chunk_max and u % chunk == 0
        assert n_claims == u // chunk * n_descs
        for i in range(desc0, desc0 + n_descs):
            t, k = descs[i]
            assert kinds[base[t] + k] == kind and units[base[t] + k] == u
        claim += n_claims
        desc += n_descs
    assert claim == sch["claims"] and desc == len(descs)
    # claims of each descriptor; every unit swept once
    claims_of = {i: [] for i in range(len(descs))}
    swept = {i: [] for i in range(len(descs))}
    for c in range(sch["claims"]):
        d, u0, n = _claim_desc(segs, c)
        claims_of[d].append(c)
        swept[d] += list(range(u0, u0 + n))
    for i, (t, k) in enumerate(descs):
        assert sorted(swept[i]) == list(range(units[base[t] + k]))
    # dependencies: the previous pass, else the parent's last pass; all of a
    # dependency's claims come before every claim that waits for it
    for i, (t, k) in enumerate(descs):
        dep, need = deps[i]
        if k > 0:
            want = pos[(t, k - 1)]
        elif parents[t] >= 0:
            want = pos[(parents[t], passes[parents[t]] - 1)]
        else:
            want = -1
        assert dep == want, (t, k)
        if dep >= 0:
            dt, dk = descs[dep]
            assert need == units[base[dt] + dk]
            assert max(claims_of[dep]) < min(claims_of[i])
    return claims_of


def _simulate(sch, workers, rng):
    """Workgroups take claims in order; a claim runs once its dependency's
    counter has reached `need`; returns the number of claims completed."""
    segs, deps = sch["segments"], sch["deps"]
    total = sch["claims"]
    counter = [0] * len(sch["descs"])
    nxt = 0
    waiting = []            # workers holding a claim whose dependency is unmet
    running = []            # (finish time, worker, claim)
    t_now = 0.0
    idle = list(range(workers))
    done = 0

    def ready(c):
        d, _, _ = _claim_desc(segs, c)
        dep, need = deps[d]
        return dep < 0 or counter[dep] >= need

    while done < total:
        # idle workers claim in order
        while idle and nxt < total:
            w = idle.pop()
            waiting.append((w, nxt))
            nxt += 1
        still = []
        for w, c in waiting:
            if ready(c):
                heapq.heappush(running, (t_now + float(rng.exponential(1.0)), w, c))
            else:
                still.append((w, c))
        waiting = still
        if not running:
            break           # nothing can progress: a deadlock
        t_now, w, c = heapq.heappop(running)
        d, _, n = _claim_desc(segs, c)
        counter[d] += n
        done += 1
        idle.append(w)
    return done, counter


@pytest.mark.parametrize("seed", range(12))
def test_random_tree_schedules(seed):
    rng = np.random.default_rng(700 + seed)
    n_tasks = int(rng.integers(1, 40))
    parents, passes, kinds, units = _random_tree(rng, n_tasks)
    chunk_max = int(2 ** rng.integers(0, 5))
    grid = int(rng.integers(1, 64))
    sch = B.persist_schedule(parents, passes, kinds, units, chunk_max, grid)
    _check_structure(sch, parents, passes, kinds, units, chunk_max, grid)
    base = np.cumsum([0] + list(passes))
    for workers in (1, 2, 7, grid, 500):
        done, counter = _simulate(sch, workers, rng)
        assert done == sch["claims"], (workers, done)
        for i, (t, k) in enumerate(sch["descs"]):
            assert counter[i] == units[base[t] + k]


def test_prefix_tree_shape():
    """Config 3's shape (8 roots, 64 children, 512 leaves of 1..7 passes):
    levels follow depth, and leaves wait for their parents' last passes."""
    rng = np.random.default_rng(3)
    parents = [-1] * 8 + [k // 8 for k in range(64)] + [8 + k // 8 for k in range(512)]
    passes = [1] * 72 + [int(rng.integers(1, 8)) for _ in range(512)]
    kinds, units = [], []
    for t in range(len(parents)):
        for k in range(passes[t]):
            kinds.append(0 if t < 72 else 1 + min(k, 6))
            units.append(64)
    sch = B.persist_schedule(parents, passes, kinds, units, 8, 256)
    _check_structure(sch, parents, passes, kinds, units, 8, 256)
    # the first level is the 8 roots in one segment, then the 64 children
    assert sch["segments"][0][2:4] == [0, 8] and sch["segments"][1][2:4] == [8, 64]
    done, _ = _simulate(sch, 256, rng)
    assert done == sch["claims"]


def test_schedule_refuses_bad_trees():
    with pytest.raises(B.QwError):
        B.persist_schedule([-1, 2, 0], [1, 1, 1], [0, 0, 0], [16, 16, 16])   # parent after child
    with pytest.raises(B.QwError):
        B.persist_schedule([-1, 0], [0, 1], [0], [16])                       # parent without passes
    with pytest.raises(B.QwError):
        B.persist_schedule([-1], [1], [0], [12])                             # units not a power of two
    with pytest.raises(B.QwError):
        B.persist_schedule([-1], [1], [0], [16], chunk_max=3)

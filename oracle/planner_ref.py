"""Reference forms of the planner's closed-form rules (TEST INFRASTRUCTURE ONLY).

* Eq. (2), Sec. IV-C: reuse a prefix shared by N tasks iff
      (N - 1) C_prefix > C_materialize + N (C_reload + C_handoff) + delta,
  with C_handoff = 0 for a same-backend continuation.
* delta: the "10 % guard" of the evaluation (Sec. V, baselines; Sec. VI Q6),
  read as delta = g * est_reuse with g = 0.10, where
      est_reuse  = C_prefix + C_materialize + N (C_reload + C_handoff + C_suffix)
      est_direct = N (C_prefix + C_suffix),
  so that Eq. (2) becomes est_direct > (1 + g) est_reuse. The threshold-0
  ablation is g = 0.
"""
from __future__ import annotations


def eq2_reuse(n_tasks: int, c_prefix: float, c_materialize: float,
              c_reload: float, c_handoff: float, delta: float) -> bool:
    return (n_tasks - 1) * c_prefix > c_materialize + n_tasks * (c_reload + c_handoff) + delta


def estimates(n_tasks: int, c_prefix: float, c_suffix: float, c_materialize: float,
              c_reload: float, c_handoff: float = 0.0):
    est_direct = n_tasks * (c_prefix + c_suffix)
    est_reuse = c_prefix + c_materialize + n_tasks * (c_reload + c_handoff + c_suffix)
    return est_direct, est_reuse


def guarded_reuse(n_tasks: int, c_prefix: float, c_suffix: float, c_materialize: float,
                  c_reload: float, c_handoff: float = 0.0, guard: float = 0.10) -> bool:
    """Eq. (2) with delta = guard * est_reuse."""
    _, est_reuse = estimates(n_tasks, c_prefix, c_suffix, c_materialize, c_reload, c_handoff)
    return eq2_reuse(n_tasks, c_prefix, c_materialize, c_reload, c_handoff, guard * est_reuse)


def break_even_tasks(c_prefix: float, c_suffix: float, c_materialize: float,
                     c_reload: float, c_handoff: float = 0.0, guard: float = 0.0,
                     n_max: int = 1 << 20) -> int:
    """Smallest N for which the guarded rule chooses reuse (0 if none <= n_max)."""
    for n in range(1, n_max + 1):
        if guarded_reuse(n, c_prefix, c_suffix, c_materialize, c_reload, c_handoff, guard):
            return n
    return 0

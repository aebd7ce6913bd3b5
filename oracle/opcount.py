"""Algorithmic operation counts of one vertex-step (oracle; test infrastructure).

The work of the reaction + SDC stage is counted as forward-mode
differentiation restricted to the compile-time Jacobian pattern (the paper's
CTSM idea, section 3.3.2): every model operation costs one operation on its
value plus the operations its derivative rule needs on the partials that are
structurally non-zero.  ``CountDual`` is a Dual whose value is one float and
whose partials are a set of state indices; running a model's rhs with it
counts, per category, the operations of

  F   -- the right-hand side alone,
  FJ  -- the right-hand side and its Jacobian on the pattern.

The static sparse solve of (I - dtau J) x = b is counted from the pattern with
the symbolic fill of the elimination order "gates first, then the dense core".
Flops: add, mul, div and every transcendental count one each (a fused
multiply-add is a mul and an add); comparisons and selects are not counted.

Run  python -m oracle.opcount  to print the per-evaluation figures.
"""
from __future__ import annotations

from collections import Counter

import numpy as np

from .ad import Dual
from .models import LR91, TT06

FLOP_KINDS = ("add", "mul", "div", "exp", "log", "sqrt", "expm1")


class CountDual(Dual):
    counts = Counter()

    def __init__(self, v, d):
        super().__init__(float(v), frozenset(d))

    @classmethod
    def tick(cls, kind, n=1):
        cls.counts[kind] += n

    def _lin(self, o, sign):
        if isinstance(o, Dual):
            self.tick("add", 1 + len(self.d & o.d))
            return CountDual(self.v + sign * o.v, self.d | o.d)
        self.tick("add")
        return CountDual(self.v + sign * o, self.d)

    def __add__(self, o):
        return self._lin(o, 1.0)

    __radd__ = __add__

    def __sub__(self, o):
        return self._lin(o, -1.0)

    def __rsub__(self, o):
        self.tick("add")
        return CountDual(o - self.v, self.d)

    def __neg__(self):
        return CountDual(-self.v, self.d)

    def __mul__(self, o):
        if isinstance(o, Dual):
            both = len(self.d & o.d)
            one = len(self.d ^ o.d)
            self.tick("mul", 1 + 2 * both + one)
            self.tick("add", both)
            return CountDual(self.v * o.v, self.d | o.d)
        self.tick("mul", 1 + len(self.d))
        return CountDual(self.v * o, self.d)

    __rmul__ = __mul__

    def __truediv__(self, o):
        if isinstance(o, Dual):
            # inv = 1/b, q = a inv; partials (x - q y) inv
            both = len(self.d & o.d)
            only_a = len(self.d - o.d)
            only_b = len(o.d - self.d)
            self.tick("div")
            self.tick("mul", 1 + 2 * both + only_a + (1 + 2 * only_b if only_b else 0))
            self.tick("add", both)
            return CountDual(self.v / o.v, self.d | o.d)
        self.tick("mul", 1 + len(self.d))
        return CountDual(self.v / o, self.d)

    def __rtruediv__(self, o):
        self.tick("div")
        self.tick("mul", 1 + (1 + len(self.d) if self.d else 0))
        return CountDual(o / self.v, self.d)

    def __pow__(self, p):
        if p == 2:
            return self * self
        if p == 3:
            return self * self * self
        raise TypeError("only squares and cubes are used by the models")

    def __ge__(self, o):
        return self.v >= (o.v if isinstance(o, Dual) else o)

    def __gt__(self, o):
        return self.v > (o.v if isinstance(o, Dual) else o)

    def __eq__(self, o):
        return self.v == (o.v if isinstance(o, Dual) else o)

    __hash__ = None

    def _exp(self):
        self.tick("exp")
        self.tick("mul", len(self.d))
        return CountDual(np.exp(self.v), self.d)

    def _expm1(self):
        self.tick("expm1")
        if self.d:
            self.tick("add")                        # exp(x) = expm1(x) + 1 for the partials
            self.tick("mul", len(self.d))
        return CountDual(np.expm1(self.v), self.d)

    def _log(self):
        self.tick("log")
        if self.d:
            self.tick("div")
            self.tick("mul", len(self.d))
        return CountDual(np.log(self.v), self.d)

    def _sqrt(self):
        self.tick("sqrt")
        if self.d:
            self.tick("div")
            self.tick("mul", 1 + len(self.d))
        return CountDual(np.sqrt(self.v), self.d)

    @staticmethod
    def _where(cond, a, b):
        cond = bool(np.all(cond))
        pick = a if cond else b
        da = a.d if isinstance(a, Dual) else frozenset()
        db = b.d if isinstance(b, Dual) else frozenset()
        v = pick.v if isinstance(pick, Dual) else float(np.asarray(pick).reshape(-1)[0])
        return CountDual(v, da | db)


class TapeDual(Dual):
    """A Dual that records every operation on a tape, with the cost of its
    value and of each of its partials, so that the work feeding a chosen set
    of outputs (values of some rows, some partials of some rows) can be
    counted.  This is what an optimising compiler keeps when an evaluation's
    consumer reads only part of the result (the Rush-Larsen evaluations).
    The per-operation costs are those of CountDual."""
    tape = []

    def __init__(self, v, d, parents=(), vcost=None, shared=None, pcost=None):
        super().__init__(float(v), frozenset(d))
        self.parents = tuple(p for p in parents if isinstance(p, TapeDual))
        self.vcost = Counter(vcost or {})
        self.shared = Counter(shared or {})      # once if any partial is needed
        self.pcost = pcost or {}                 # partial index -> Counter
        self.id = len(TapeDual.tape)
        TapeDual.tape.append(self)

    def _lin(self, o, sign):
        if isinstance(o, Dual):
            both = self.d & o.d
            return TapeDual(self.v + sign * o.v, self.d | o.d, (self, o), {"add": 1},
                            pcost={k: {"add": 1} for k in both})
        return TapeDual(self.v + sign * o, self.d, (self,), {"add": 1})

    def __add__(self, o):
        return self._lin(o, 1.0)

    __radd__ = __add__

    def __sub__(self, o):
        return self._lin(o, -1.0)

    def __rsub__(self, o):
        return TapeDual(o - self.v, self.d, (self,), {"add": 1})

    def __neg__(self):
        return TapeDual(-self.v, self.d, (self,))

    def __mul__(self, o):
        if isinstance(o, Dual):
            both = self.d & o.d
            pc = {k: ({"mul": 2, "add": 1} if k in both else {"mul": 1}) for k in self.d | o.d}
            return TapeDual(self.v * o.v, self.d | o.d, (self, o), {"mul": 1}, pcost=pc)
        return TapeDual(self.v * o, self.d, (self,), {"mul": 1},
                        pcost={k: {"mul": 1} for k in self.d})

    __rmul__ = __mul__

    def __truediv__(self, o):
        if isinstance(o, Dual):
            both, only_a, only_b = self.d & o.d, self.d - o.d, o.d - self.d
            pc = {}
            for k in both:
                pc[k] = {"mul": 2, "add": 1}
            for k in only_a:
                pc[k] = {"mul": 1}
            for k in only_b:
                pc[k] = {"mul": 2}
            return TapeDual(self.v / o.v, self.d | o.d, (self, o), {"div": 1, "mul": 1},
                            shared={"mul": 1} if only_b else None, pcost=pc)
        return TapeDual(self.v / o, self.d, (self,), {"mul": 1},
                        pcost={k: {"mul": 1} for k in self.d})

    def __rtruediv__(self, o):
        return TapeDual(o / self.v, self.d, (self,), {"div": 1, "mul": 1}, shared={"mul": 1},
                        pcost={k: {"mul": 1} for k in self.d})

    def __pow__(self, p):
        if p == 2:
            return self * self
        if p == 3:
            return self * self * self
        raise TypeError("only squares and cubes are used by the models")

    def __ge__(self, o):
        return self.v >= (o.v if isinstance(o, Dual) else o)

    def __gt__(self, o):
        return self.v > (o.v if isinstance(o, Dual) else o)

    def __le__(self, o):
        return self.v <= (o.v if isinstance(o, Dual) else o)

    def __lt__(self, o):
        return self.v < (o.v if isinstance(o, Dual) else o)

    def __eq__(self, o):
        return self.v == (o.v if isinstance(o, Dual) else o)

    __hash__ = None

    def _exp(self):
        return TapeDual(np.exp(self.v), self.d, (self,), {"exp": 1},
                        pcost={k: {"mul": 1} for k in self.d})

    def _expm1(self):
        return TapeDual(np.expm1(self.v), self.d, (self,), {"expm1": 1}, shared={"add": 1},
                        pcost={k: {"mul": 1} for k in self.d})

    def _log(self):
        return TapeDual(np.log(self.v), self.d, (self,), {"log": 1}, shared={"div": 1},
                        pcost={k: {"mul": 1} for k in self.d})

    def _sqrt(self):
        return TapeDual(np.sqrt(self.v), self.d, (self,), {"sqrt": 1},
                        shared={"div": 1, "mul": 1}, pcost={k: {"mul": 1} for k in self.d})

    @staticmethod
    def _where(cond, a, b):
        cond = bool(np.all(cond))
        pick = a if cond else b
        da = a.d if isinstance(a, Dual) else frozenset()
        db = b.d if isinstance(b, Dual) else frozenset()
        v = pick.v if isinstance(pick, Dual) else float(np.asarray(pick).reshape(-1)[0])
        return TapeDual(v, da | db, (a, b))


def needed_work(model, x, seeds, rows_value, rows_partials, i_stim=-10.0, i_diff=0.3):
    """Flops of one evaluation seeded on the states `seeds` when only the values
    of rows `rows_value` and, for rows `rows_partials`, the partials with respect
    to the seeded states are used.  Backward reachability over the tape: a
    needed value needs its operands' values; a needed partial k needs the
    operands' partials k and every operand value (the derivative rules use them)."""
    TapeDual.tape = []
    xs = [TapeDual(v, {i} if i in seeds else ()) for i, v in enumerate(x)]
    out = model._rhs(xs, i_stim, i_diff, model.params, False)
    tape = TapeDual.tape
    need_v = [False] * len(tape)
    need_p = [set() for _ in tape]
    for i in rows_value:
        if isinstance(out[i], TapeDual):
            need_v[out[i].id] = True
    for i in rows_partials:
        if isinstance(out[i], TapeDual):
            need_p[out[i].id] |= set(out[i].d)
    for node in reversed(tape):
        nid = node.id
        if need_p[nid]:
            need_v[nid] = True
        if need_v[nid]:
            for par in node.parents:
                need_v[par.id] = True
        for k in need_p[nid]:
            for par in node.parents:
                if k in par.d:
                    need_p[par.id].add(k)
    total = Counter()
    for node in tape:
        if need_v[node.id]:
            total.update(node.vcost)
        if need_p[node.id]:
            total.update(node.shared)
            for k in need_p[node.id]:
                total.update(node.pcost.get(k, {}))
    return flops(total)


def core_solve_flops(pattern, n_core):
    """Flops of the dense-on-pattern elimination of the core block alone."""
    core = [[k for k in row if k < n_core] for row in pattern[:n_core]]
    return solve_flops(core, n_core)[0]


def rush_larsen_counts(model, x, n_core):
    """Per-evaluation work of the Rush-Larsen predictor: the gating-state
    evaluation (every row's value, for F(X_n); or the gating rows' values only,
    on later sub-intervals) with the gating rows' own partials, and one core
    Newton evaluation (core rows' values and partials on the core)."""
    n = model.n
    gating = list(range(n_core, n))
    core = list(range(n_core))
    return {
        "gate_step_first": needed_work(model, x, set(gating), range(n), gating),
        "gate_step": needed_work(model, x, set(gating), gating, gating),
        "core_FJ": needed_work(model, x, set(core), core, core),
        "core_solve": core_solve_flops(count_eval(model, x, True)[1], n_core),
    }


def count_eval(model, x, with_jacobian, i_stim=-10.0, i_diff=0.3):
    """Operation counts of one F (or F and J) evaluation at state x."""
    CountDual.counts = Counter()
    xs = [CountDual(v, {i} if with_jacobian else ()) for i, v in enumerate(x)]
    out = model._rhs(xs, i_stim, i_diff, model.params, False)
    pattern = [sorted(o.d) if isinstance(o, Dual) else [] for o in out]
    return dict(CountDual.counts), pattern


def solve_flops(pattern, n_fp64):
    """Flops of the static elimination: gates (states n_fp64..n-1) first, then the core."""
    n = len(pattern)
    P = np.zeros((n, n), dtype=bool)
    for i, row in enumerate(pattern):
        P[i, row] = True
        P[i, i] = True
    order = list(range(n_fp64, n)) + list(range(n_fp64))
    flops = 0
    for k, p in enumerate(order):
        flops += 1                                  # reciprocal of the pivot
        later = order[k + 1:]
        for i in later:
            if not P[i, p]:
                continue
            flops += 1                              # l = a_ip / a_pp
            for j in later:
                if P[p, j]:
                    P[i, j] = True
                    flops += 2                      # a_ij -= l a_pj
            flops += 2                              # b_i -= l b_p
    for k, p in enumerate(order):
        flops += 2 * int(sum(P[p, j] for j in order[k + 1:])) + 1
    return flops, int(P.sum())


def resolve_flops(pattern, n_fp64):
    """Flops of a second right-hand side on a kept factorisation (ROS2 stage 2):
    forward substitution with the multipliers and back substitution on the
    filled pattern, gates first as in solve_flops."""
    n = len(pattern)
    P = np.zeros((n, n), dtype=bool)
    for i, row in enumerate(pattern):
        P[i, row] = True
        P[i, i] = True
    order = list(range(n_fp64, n)) + list(range(n_fp64))
    flops = 0
    for k, p in enumerate(order):
        later = order[k + 1:]
        for i in later:
            if P[i, p]:
                for j in later:
                    if P[p, j]:
                        P[i, j] = True
                flops += 2                          # b_i -= l b_p
    for k, p in enumerate(order):
        flops += 2 * int(sum(P[p, j] for j in order[k + 1:])) + 1
    return flops


def flops(c):
    return sum(c.get(k, 0) for k in FLOP_KINDS)


def per_evaluation(model, x, n_fp64):
    cF, _ = count_eval(model, x, False)
    cFJ, pattern = count_eval(model, x, True)
    sf, nnz = solve_flops(pattern, n_fp64)
    return {
        "F": flops(cF), "FJ": flops(cFJ), "solve": sf, "resolve": resolve_flops(pattern, n_fp64),
        "nnz": sum(len(r) for r in pattern),
        "nnz_filled": nnz,
        "transcendental_F": sum(cF.get(k, 0) for k in ("exp", "log", "sqrt", "expm1")),
        "div_F": cF.get("div", 0),
        "F_detail": cF, "FJ_detail": cFJ,
    }


def flops_per_launch(ev, n, n_steps, M, K, newton_iters):
    """Algorithmic flops of one launch from the evaluation counts and the Newton
    iterations the launch actually took (the library's statistics)."""
    """n: states per vertex; n_steps: vertex-steps of the launch; newton_iters: total
    Newton iterations of the launch."""
    F_evals = n_steps * K * (M - 2)   # F(X_n) comes from the first Newton evaluation
    FJ = newton_iters + n_steps * K * (M - 1)   # each Newton iteration and each sweep node
    return (F_evals * ev["F"] + FJ * (ev["FJ"] + ev["solve"])
            # Newton residual (3 flops), update and stop test (3 flops) per state
            + newton_iters * 6 * n
            # sweep: quadrature (2 flops per term), residual (2) and update (1) per state
            + n_steps * K * ((M - 1) * M * 2 + (M - 1) * 3) * n)


def flops_per_launch_rl(ev, rl, n, n_core, n_steps, M, K, newton_iters):
    """Algorithmic flops of one launch with the Rush-Larsen predictor: per step
    the gating-state evaluation of every sub-interval (the first also gives
    F(X_n)), 7 flops per gating state for its exponential step, and per core
    Newton iteration the core evaluation, the core solve and 6 flops per core
    state; the sweeps as with the other predictors."""
    gates = n - n_core
    per_step = rl["gate_step_first"] + (M - 2) * rl["gate_step"] + (M - 1) * 7 * gates
    sweeps = (K * (M - 2) * ev["F"] + K * (M - 1) * (ev["FJ"] + ev["solve"])
              + K * ((M - 1) * M * 2 + (M - 1) * 3) * n)
    return (n_steps * (per_step + sweeps)
            + newton_iters * (rl["core_FJ"] + rl["core_solve"] + 6 * n_core))


def flops_per_launch_ros2(ev, n, n_steps, M, K):
    """Algorithmic flops of one launch with the ROS2 predictor: per sub-interval
    one F+J evaluation with its elimination, one F evaluation and one second
    solve, plus the stage arithmetic per state (stage-1 right-hand side 1, stage
    point 2, stage-2 right-hand side 2, update 4, error estimate 3); the sweeps
    as with the Newton predictor except that F(X_n) comes from the first stage."""
    per_sub = ev["FJ"] + ev["solve"] + ev["F"] + ev["resolve"] + 12 * n
    sweeps = (K * (M - 2) * ev["F"] + K * (M - 1) * (ev["FJ"] + ev["solve"])
              + K * ((M - 1) * M * 2 + (M - 1) * 3) * n)
    return n_steps * ((M - 1) * per_sub + sweeps)


if __name__ == "__main__":
    from . import rest, tt06
    for model, x, n64 in ((LR91, rest.lr91_rest(), 2), (TT06, tt06.published_initial(), 6)):
        ev = per_evaluation(model, x, n64)
        print(model.name, {k: v for k, v in ev.items() if not k.endswith("detail")})
        print("   F:", ev["F_detail"])
        print("   FJ:", ev["FJ_detail"])
        print("   Rush-Larsen:", rush_larsen_counts(model, x, n64))

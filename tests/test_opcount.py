"""The flop constants bench.py uses equal what the oracle's op counter
computes, and the counter itself counts sensibly (F+J costs more than F,
the solve count follows the pattern's fill)."""
import importlib.util
import os

from oracle import rest, tt06
from oracle.models import LR91, TT06
from oracle.opcount import per_evaluation, solve_flops

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_bench_constants_match_the_counter():
    b = _bench()
    for model, x, n64, const in ((TT06, tt06.published_initial(), 6, b.TT06_FLOPS),
                                 (LR91, rest.lr91_rest(), 2, b.LR91_FLOPS)):
        ev = per_evaluation(model, x, n64)
        assert {k: ev[k] for k in ("F", "FJ", "solve", "resolve")} == const, model.name
        assert ev["resolve"] < ev["solve"]
        assert ev["FJ"] > ev["F"]
    assert per_evaluation(TT06, tt06.published_initial(), 6)["nnz"] == 76


def test_solve_count_on_a_tiny_pattern():
    # 2x2 dense core, one gate depending on V (state 0): gate eliminated first
    pattern = [[0, 1, 2], [0, 1], [0, 2]]
    flops, nnz = solve_flops(pattern, 2)
    # gate pivot: rcp; V row: l, a_VV update (2), b_V update (2); core: V pivot rcp, Cai row
    # l + 1 update(2)+b(2), Cai pivot rcp; back substitution: 3 rows
    assert nnz == 7
    assert flops == (1 + 1 + 2 + 2) + (1 + 1 + 2 + 2) + 1 + (2 * 1 + 1) + (2 * 0 + 1) + (2 * 1 + 1)


def test_resolve_count_on_a_tiny_pattern():
    from oracle.opcount import resolve_flops
    # same pattern as above: forward b updates (gate into V: 2; V into Cai: 2), back
    # substitution 3 rows (2 * upper entries + 1)
    pattern = [[0, 1, 2], [0, 1], [0, 2]]
    assert resolve_flops(pattern, 2) == 2 + 2 + (2 * 1 + 1) + (2 * 0 + 1) + (2 * 1 + 1)


def test_bench_launch_formulas_match_the_counter():
    from oracle.opcount import flops_per_launch, flops_per_launch_ros2
    b = _bench()
    ev = b.TT06_FLOPS
    for M, K in ((2, 1), (3, 3), (4, 2)):
        assert b.flops_per_launch_ros2(ev, 19, 1000, M, K) == flops_per_launch_ros2(ev, 19, 1000, M, K)
        assert b.flops_per_launch(ev, 19, 1000, M, K, 2500) == flops_per_launch(ev, 19, 1000, M, K, 2500)


def test_tape_counter_reproduces_the_full_counts():
    from oracle.opcount import needed_work
    for model, x, n64 in ((TT06, tt06.published_initial(), 6), (LR91, rest.lr91_rest(), 2)):
        ev = per_evaluation(model, x, n64)
        n = model.n
        assert needed_work(model, x, set(), range(n), []) == ev["F"]
        assert needed_work(model, x, set(range(n)), range(n), range(n)) == ev["FJ"]
        # fewer outputs never cost more
        assert needed_work(model, x, set(range(n64)), range(n64), range(n64)) < ev["FJ"]


def test_bench_rush_larsen_constants_and_formula():
    from oracle.opcount import flops_per_launch_rl, rush_larsen_counts
    b = _bench()
    assert rush_larsen_counts(TT06, tt06.published_initial(), 6) == b.TT06_RL_FLOPS
    for M, K in ((2, 1), (3, 3)):
        assert (b.flops_per_launch_rl(b.TT06_FLOPS, b.TT06_RL_FLOPS, 19, 6, 1000, M, K, 2400)
                == flops_per_launch_rl(b.TT06_FLOPS, b.TT06_RL_FLOPS, 19, 6, 1000, M, K, 2400))


def test_bench_kind_counts_and_split():
    """The per-kind counts behind the t_min split equal the counter's, and the
    split of a launch partitions the algorithmic count exactly (every flop is
    assigned to one unit: W64, W32 or the transcendental unit)."""
    b = _bench()
    ev = per_evaluation(TT06, tt06.published_initial(), 6)
    assert ev["F_detail"] == b.TT06_KINDS["F"]
    assert ev["FJ_detail"] == b.TT06_KINDS["FJ"]
    for M, K, it in ((3, 3, 2400), (4, 3, 3100), (2, 1, 1000)):
        vs = 1000
        total = b.flops_per_launch(b.TT06_FLOPS, 19, vs, M, K, it)
        f = b.work_split(vs, M, K, it, "fp64")
        assert f["W32"] == 0 and f["W64"] + f["Wtr"] == total
        assert f["Wtr"] == (vs * K * (M - 2) * 57 + (it + vs * K * (M - 1)) * 57)
        m = b.work_split(vs, M, K, it, "mixed")
        assert m["W64"] + m["W32"] + m["Wtr"] == total
        assert m["Wtr"] > f["Wtr"]          # divisions, sqrt and pivot reciprocals join

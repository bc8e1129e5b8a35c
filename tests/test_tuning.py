"""Host logic of the tuned planner (zpl_plan_forms touches no device).

The form choice never changes results (GPU tests check that every form gives
the same bits); these tests check which form the planner picks: the built-in
rule, the cheapest eligible form under a table, bilinear interpolation in
(alpha, ln n), eligibility limits, fallbacks and table validation.
"""
import math

import pytest

from paper_1305_6738_amd import ZplError, cell_array, load_tuning, plan_forms, save_tuning
from inputs import table_slice


# Tuned choices below are per-replicate comparisons: cells of many replicates,
# for which the soonest-finishing form is the cheapest one per replicate.
R = 10 ** 6


def grid(alphas, ns, cost):
    return [{"alpha": a, "n": n, "ns_per_replicate": list(cost(a, n))} for a in alphas for n in ns]


def test_builtin_rule_on_table_slice():
    # n = 1000: expected overflow of the per-lane list, n * P(X > 48), is at
    # most 2 from alpha = 2.5 up (lane form); below, the wave form.
    forms = plan_forms(table_slice(n=1000, R=1000))
    assert forms == ["wave"] * 4 + ["lane"] * 5


def test_builtin_rule_heavy_for_large_overflow():
    # alpha = 1.2, n = 1e4: about 1,700 values above the wave form's 1024-bin
    # histogram, more than its LDS overflow area holds
    assert plan_forms([(1.2, 10000, 10, 1, 0)]) == ["heavy"]
    assert plan_forms([(3.5, 10, 10, 1, 0)]) == ["lane"]
    assert plan_forms([(3.5, 100000, 10, 1, 0)]) == ["wave"]  # lane form needs n <= 65535


def test_table_picks_cheapest_form():
    cells = [(2.5, 100, R, 1, 0), (3.0, 1000, R, 1, 1)]
    heavy = grid([2.0, 3.5], [10, 10000], lambda a, n: (9.0, 9.0, 1.0))
    wave = grid([2.0, 3.5], [10, 10000], lambda a, n: (9.0, 1.0, 5.0))
    lane = grid([2.0, 3.5], [10, 10000], lambda a, n: (1.0, 2.0, 5.0))
    assert plan_forms(cells, heavy) == ["heavy", "heavy"]
    assert plan_forms(cells, wave) == ["wave", "wave"]
    assert plan_forms(cells, lane) == ["lane", "lane"]


def test_table_respects_eligibility():
    # lane cheapest everywhere, but at alpha = 1.5, n = 4000 a replicate has
    # about 440 values above 48 (lane ineligible: 128 slots) and about 96
    # above 1024 (wave eligible: 248 entries); at n = 1e4, about 240 above
    # 1024 (wave ineligible too)
    t = grid([1.5, 3.5], [10, 100000], lambda a, n: (1.0, 2.0, 3.0))
    assert plan_forms([(1.5, 4000, R, 1, 0)], t) == ["wave"]
    assert plan_forms([(1.5, 10000, R, 1, 0)], t) == ["heavy"]
    assert plan_forms([(1.2, 10000, R, 1, 0)], t) == ["heavy"]
    assert plan_forms([(3.0, 70000, R, 1, 0)], t) == ["wave"]  # n > 65535


def test_bilinear_interpolation_in_log_n():
    # lane cost rises from 1 at n = 100 to 100 at n = 10,000, wave is 40
    # throughout: lane wins below ln-interpolated crossover
    # w = (40 - 1) / 99 of the way from ln 100 to ln 10,000
    t = grid([3.0, 3.5], [100, 10000], lambda a, n: (1.0 if n == 100 else 100.0, 40.0, 1000.0))
    w = 39.0 / 99.0
    n_cross = math.exp(math.log(100) + w * (math.log(10000) - math.log(100)))
    below, above = int(n_cross * 0.95), int(n_cross * 1.05)
    assert plan_forms([(3.2, below, R, 1, 0)], t) == ["lane"]
    assert plan_forms([(3.2, above, R, 1, 0)], t) == ["wave"]


def test_bilinear_interpolation_in_alpha():
    # wave cost 10 at alpha 2.5, 30 at 3.5; lane cost 20 throughout:
    # crossover at alpha = 3.0
    t = grid([2.5, 3.5], [10, 1000], lambda a, n: (20.0, 10.0 if a == 2.5 else 30.0, 1000.0))
    assert plan_forms([(2.9, 500, R, 1, 0)], t) == ["wave"]
    assert plan_forms([(3.1, 500, R, 1, 0)], t) == ["lane"]


def test_clamped_outside_grid():
    t = grid([2.5, 3.0], [100, 1000], lambda a, n: (1.0, 2.0, 3.0) if a == 3.0 else (2.0, 1.0, 3.0))
    # alpha above the grid takes the last row (lane cheapest), below the first (wave)
    assert plan_forms([(3.4, 300, R, 1, 0)], t) == ["lane"]
    assert plan_forms([(2.0, 300, R, 1, 0)], t) == ["wave"]


def test_unmeasured_corner_excludes_form():
    # lane unmeasured (-1) at one corner of the cell's square: lane not chosen
    def cost(a, n):
        return (-1.0 if (a == 3.5 and n == 1000) else 1.0, 2.0, 3.0)
    t = grid([2.5, 3.5], [100, 1000], cost)
    assert plan_forms([(3.0, 300, R, 1, 0)], t) == ["wave"]
    assert plan_forms([(2.5, 100, R, 1, 0)], t) == ["lane"]


def test_all_unmeasured_falls_back_to_builtin():
    t = grid([2.5, 3.5], [100, 1000], lambda a, n: (-1.0, -1.0, -1.0))
    cells = table_slice(n=1000, R=10)
    assert plan_forms(cells, t) == plan_forms(cells)


@pytest.mark.parametrize("bad", ["not_grid", "alpha_order", "n_order", "nan", "alpha_range"])
def test_invalid_tables_rejected(bad):
    t = grid([2.5, 3.5], [100, 1000], lambda a, n: (1.0, 2.0, 3.0))
    if bad == "not_grid":
        t = t[:3]
    elif bad == "alpha_order":
        t = grid([3.5, 2.5], [100, 1000], lambda a, n: (1.0, 2.0, 3.0))
    elif bad == "n_order":
        t = grid([2.5, 3.5], [1000, 100], lambda a, n: (1.0, 2.0, 3.0))
    elif bad == "nan":
        t[1]["ns_per_replicate"][2] = float("nan")
    elif bad == "alpha_range":
        t = grid([0.5, 3.5], [100, 1000], lambda a, n: (1.0, 2.0, 3.0))
    with pytest.raises(ZplError) as e:
        plan_forms([(3.0, 300, R, 1, 0)], t)
    assert e.value.status == -1


def test_save_load_roundtrip(tmp_path):
    t = grid([2.5, 3.5], [100, 1000], lambda a, n: (a * n, -1.0, 0.125))
    p = tmp_path / "tune.json"
    save_tuning(p, t)
    assert load_tuning(p) == t
    cells = [(3.0, 300, 10, 1, 0), (2.6, 150, 10, 1, 1)]
    assert plan_forms(cells, load_tuning(p)) == plan_forms(cells, t)


def test_truncated_cells_plan_and_validate():
    # on 1..20 no value exceeds the lane form's 48-bin column: always lane
    assert plan_forms([(0.25, 5000, 10, 1, 0, 20), (4.0, 10, 10, 1, 1, 20)]) == ["lane", "lane"]
    # on 1..4096 with g = 0.25 most values exceed 1024: neither lane nor wave
    assert plan_forms([(0.25, 10000, 10, 1, 0, 4096)]) == ["heavy"]
    # the truncated law admits g <= 1 (and g <= 0)
    assert plan_forms([(-0.5, 100, 10, 1, 0, 50)])[0] in ("lane", "wave", "heavy")
    for bad in [(1.5, 10, 10, 1, 0, 1), (1.5, 10, 10, 1, 0, 4097), (-65.0, 10, 10, 1, 0, 20),
                (0.5, 10, 10, 1, 0, 0)]:
        with pytest.raises(ZplError) as e:
            plan_forms([bad])
        assert e.value.status == -1, bad


def test_truncated_cells_ignore_the_pure_law_table():
    """A table measures the pure law only: under one that makes the heavy
    form cheapest everywhere, truncated cells keep the built-in rule (the
    heavy form runs their K-term sums one replicate per wave), and pure cells
    beside them follow the table."""
    heavy = grid([1.5, 3.5], [10, 100000], lambda a, n: (9.0, 9.0, 1.0))
    cells = [(0.25, 50000, R, 1, 0, 1000), (4.0, 20000, R, 1, 1, 20), (1.0, 10, R, 1, 2, 1000),
             (2.5, 1000, R, 1, 3)]
    assert plan_forms(cells, heavy) == plan_forms(cells[:3]) + ["heavy"]
    assert plan_forms(cells[:3], heavy) == ["wave", "lane", "wave"]


def test_few_long_replicates_spread_over_the_device():
    """A bootstrap-sized cell (2,500 replicates of 98,000 draws): the wave
    form is cheaper per replicate (208 against 545 ns with the device busy)
    but puts 2,500 replicates in 5 workgroups, one round of about 27 ms; the
    heavy form's 313 units of 8 fit in one round of about 2.2 ms."""
    t = grid([2.5, 3.0], [10000, 100000], lambda a, n: (-1.0, 208.0, 545.0))
    assert plan_forms([(2.65, 98000, 2500, 1, 0)], t) == ["heavy"]
    assert plan_forms([(2.65, 98000, 10 ** 6, 1, 0)], t) == ["wave"]


def test_cell_array_is_taken_as_it_is():
    # a converted zpl_cell array passes through unchanged and plans the same
    cells = table_slice(n=1000, R=1000) + [{"alpha": 1.3, "n": 10**4, "replicates": 5}]
    arr = cell_array(cells)
    assert cell_array(arr) is arr
    assert len(arr) == len(cells)
    assert arr[-1].alpha == 1.3 and arr[-1].n == 10**4 and arr[-1].replicates == 5
    assert plan_forms(arr) == plan_forms(cells)

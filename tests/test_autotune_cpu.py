"""The autotuner's coordinate descent on the CPU, with a synthetic cost in
place of timing batches on the GPU."""
import pytest

from paper_2204_12876_amd import autotune as at

SPACE = {"a": [1, 2, 4, 8], "b": [16, 32, 64], "c": [0, 1]}
START = {"a": 1, "b": 16, "c": 0}


def _fake_timer(cost, calls):
    def time_tuning(run_batch, tuning, reps=8, repeats=3, device=None):
        calls.append(dict(tuning))
        return cost(tuning)
    return time_tuning


def test_descent_finds_the_optimum_of_a_separable_cost(monkeypatch):
    # the best value of each knob does not depend on the others
    cost = lambda t: 1.0 + (t["a"] - 4) ** 2 + 0.01 * abs(t["b"] - 32) + 0.5 * t["c"]
    calls = []
    monkeypatch.setattr(at, "time_tuning", _fake_timer(cost, calls))
    best, best_t, hist = at.autotune(None, START, space=SPACE)
    assert best == {"a": 4, "b": 32, "c": 0}
    assert best_t == cost(best)
    # the history holds the start and every candidate timed, in order
    assert hist[0] == (START, cost(START))
    assert [h[0] for h in hist] == calls
    # the first knob's candidates are its other values, the rest held at the start
    assert calls[1:4] == [dict(START, a=2), dict(START, a=4), dict(START, a=8)]


def test_descent_keeps_only_clear_wins(monkeypatch):
    # a 1% gain is noise: the start is kept and the search stops after one round
    cost = lambda t: 1.0 - 0.01 * (t["a"] == 8)
    calls = []
    monkeypatch.setattr(at, "time_tuning", _fake_timer(cost, calls))
    best, best_t, hist = at.autotune(None, START, space=SPACE)
    assert best == START and best_t == 1.0
    n_round = sum(len(v) - 1 for v in SPACE.values())
    assert len(calls) == 1 + n_round


def test_descent_repeats_until_a_round_changes_nothing(monkeypatch):
    # coupled knobs: b's best value moves once a has moved, so a second round is needed
    cost = lambda t: 1.0 + (t["a"] - 8) ** 2 + (t["b"] - 8 * t["a"]) ** 2 / 100.0
    calls = []
    monkeypatch.setattr(at, "time_tuning", _fake_timer(cost, calls))
    best, _, _ = at.autotune(None, START, space=SPACE, max_rounds=3)
    assert best["a"] == 8 and best["b"] == 64
    n_round = sum(len(v) - 1 for v in SPACE.values())
    assert len(calls) >= 1 + 2 * n_round


@pytest.mark.parametrize("knob", sorted(at.SPACE))
def test_search_space_holds_valid_values(knob):
    vals = at.SPACE[knob]
    assert vals == sorted(set(vals))
    if knob == "seg":
        assert all(1 <= v <= 255 for v in vals)          # the library's segment range
    else:
        assert all(1 <= v <= 65536 for v in vals)        # the library's grid range

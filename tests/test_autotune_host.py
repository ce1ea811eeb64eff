"""The autotuner's search on the CPU, with the timed trial replaced by a
cost function: coordinate descent reaches the best configuration of a
separable cost, tunes each knob only where it can matter, runs no
configuration twice, and refuses a configuration that changes the
results."""
import types

import numpy as np
import pytest

from paper_cs_0105004_amd import autotune as A
from paper_cs_0105004_amd import scenarios as S


def scen(lane_change=False, short=False):
    lens = np.array([6 if short else 40, 50], np.int32)
    return types.SimpleNamespace(flags=S.FLAG_LANE_CHANGE if lane_change else 0,
                                 link_len=lens, vmax=5, ring=False)


def fake_trials(monkeypatch, cost, hashes=lambda cfg: (1,)):
    calls = []

    def trial(scens, cfg, warm, steps, reps):
        calls.append(dict(cfg))
        return {**cfg, "us_per_step": cost(cfg), "hashes": hashes(cfg)}

    monkeypatch.setattr(A, "_trial", trial)
    return calls


def separable(cfg):
    return (abs(np.log2(cfg["tile_lanes"] / 32)) +
            abs(np.log2(cfg["tile_cells"] / 8192)) +
            abs(np.log2(cfg["back_pieces"] / 2)) +
            abs(np.log2(cfg["graph_steps"] / 128)) + 1.0)


def test_descent_finds_the_best_of_a_separable_cost(monkeypatch):
    calls = fake_trials(monkeypatch, separable)
    best = A.autotune([scen()])  # one scenario, one kernel per step
    assert (best["tile_lanes"], best["tile_cells"], best["graph_steps"]) == (32, 8192, 128)
    # back_pieces stays at 4 (untuned here), which costs 1 above the optimum
    assert best["us_per_step"] == 2.0
    keys = [tuple(sorted(c.items())) for c in calls]
    assert len(keys) == len(set(keys))  # no configuration is run twice
    assert {c["back_pieces"] for c in calls} == {4}  # not a two-kernel slot


def test_knobs_only_where_they_matter(monkeypatch):
    calls = fake_trials(monkeypatch, separable)
    best = A.autotune([scen(lane_change=True)])  # one two-kernel scenario
    assert {c["tile_cells"] for c in calls} == {2048}
    assert best["back_pieces"] == 2
    calls = fake_trials(monkeypatch, separable)
    A.autotune([scen(lane_change=True), scen(short=True)])  # a batch
    assert {c["back_pieces"] for c in calls} == {1}
    assert {c["tile_cells"] for c in calls} == {2048}
    calls = fake_trials(monkeypatch, separable)
    A.autotune([scen(), scen(lane_change=True)])  # a batch with a one-kernel slot
    assert len({c["tile_cells"] for c in calls}) == len(A.TILE_CELLS)


def test_a_configuration_that_changes_results_is_an_error(monkeypatch):
    fake_trials(monkeypatch, separable,
                hashes=lambda cfg: (2,) if cfg["tile_lanes"] == 64 else (1,))
    with pytest.raises(RuntimeError, match="changed the results"):
        A.autotune([scen()])


def test_no_scenarios(monkeypatch):
    fake_trials(monkeypatch, separable)
    with pytest.raises(ValueError):
        A.autotune([])

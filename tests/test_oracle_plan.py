"""Pins of the partitioner reference against the paper's printed facts."""
import json
import os

import pytest

from oracle import plan_ref

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def test_worked_example():
    g = _load("partition_worked_example.json")
    assert g["M"] * g["K"] + g["K"] * g["N"] + g["M"] * g["N"] == g["total_elems"]
    h, w = plan_ref.partition(g["M"], g["N"], g["K"], g["budget_elems"])
    assert (h, w) == (g["h"], g["w"])
    assert h * w == g["blocks"]
    assert plan_ref.footprint(g["M"], g["N"], g["K"], h, w) <= g["budget_elems"]
    # the whole problem does not fit (that is why it is split)
    assert plan_ref.footprint(g["M"], g["N"], g["K"], 1, 1) > g["budget_elems"]


def test_incore_thresholds():
    g = _load("incore_thresholds.json")
    for case in g["cases"]:
        n = plan_ref.max_incore_square(case["mem_bytes"], step=g["step"])
        assert n == case["max_incore_N"], case
        e = case["mem_bytes"] // 8
        assert plan_ref.partition(n, n, n, e) == (1, 1)
        m = n + g["step"]
        assert plan_ref.partition(m, m, m, e) != (1, 1)


def test_search_matches_bruteforce_small():
    for M in (1, 2, 3, 5, 8):
        for N in (1, 2, 4, 7):
            for K in (1, 3, 8):
                for budget in range(3, 3 * (M * K + K * N + M * N) + 2, 3):
                    assert plan_ref.partition(M, N, K, budget) == plan_ref.partition_bruteforce(M, N, K, budget), (M, N, K, budget)


def test_chosen_plan_is_minimal_and_fits():
    for (M, N, K, budget) in [(1024, 1024, 1024, (8 << 20) // 8), (32768, 32768, 32768, (4 << 30) // 8),
                              (65536, 16384, 32768, (8 << 30) // 8), (262144, 8192, 8192, (2 << 30) // 8)]:
        h, w = plan_ref.partition(M, N, K, budget)
        assert plan_ref.footprint(M, N, K, h, w) <= budget
        # no split with fewer B slices fits at any h
        for w2 in range(1, w):
            assert all(plan_ref.footprint(M, N, K, hh, w2) > budget for hh in (1, M))
        if h > 1:
            assert plan_ref.footprint(M, N, K, h - 1, w) > budget


def test_infeasible_returns_none():
    assert plan_ref.partition(4, 4, 8, 10) is None

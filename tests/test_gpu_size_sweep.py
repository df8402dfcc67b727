"""Throughput and results across the in-core / out-of-core boundary (Section
VI): at the paper's largest in-core size for a 12 GiB device (N = 22528) the
paper's partitioner runs the product in core, at the next size of its sweep
(24576) out of core; the end-to-end rate must not drop across the switch, for
the paper's partitioner and for the cost model, and every product of the two
sizes is checked against the oracle on sampled rows."""
import numpy as np
import pytest

from gpu_helpers import sample_rows, gate_errors
import oracle
from paper_1808_05056_amd import size_sweep as S

pytestmark = pytest.mark.gpu
GiB = 1 << 30


def _check(name, w, A, B, C, plan):
    # beta = 0: C is not read, so the reference needs no initial C
    rows = sample_rows(w.M, plan.mb, count=64, seed=w.M)
    ref, D = oracle.gemm_rows(w.alpha, A, B, 0.0, None, rows=rows)
    gate_errors(C[rows], ref, w.alpha, D, 0.0, None, label=f"N={w.M} {name} {len(rows)} rows: ")


def test_no_loss_across_the_in_core_limit():
    budget = 12 * GiB
    below = S.measure(22528, budget, reps=2, check=_check)
    above = S.measure(24576, budget, reps=2, check=_check)
    for name in ("paper", "model"):
        print(f"{name}: N=22528 {below[name][2]:.2f} TFLOP/s {below[name][0]}; "
              f"N=24576 {above[name][2]:.2f} TFLOP/s {above[name][0]}", flush=True)
    assert S.is_in_core(below["paper"][0], 22528)
    assert not S.is_in_core(above["paper"][0], 24576)
    for name in ("paper", "model"):
        assert above[name][2] >= 0.95 * below[name][2], name

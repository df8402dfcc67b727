"""Shared pieces of the GPU tests: page-locked workload matrices filled from the
seeded generator, sampled-row selection and the comparison against the CPU
reference (which regenerates the initial C rows it needs)."""
import numpy as np

import oracle
import synth
import paper_1808_05056_amd as ooc


class PinnedProblem:
    """A, B, C of a workload in page-locked host memory."""

    def __init__(self, w, ld_pad=(0, 0, 0), nan_c=False):
        self.w = w
        self.Am = ooc.PinnedMatrix(w.M, w.K, w.K + ld_pad[0])
        self.Bm = ooc.PinnedMatrix(w.K, w.N, w.N + ld_pad[1])
        self.Cm = ooc.PinnedMatrix(w.M, w.N, w.N + ld_pad[2])
        self.A, self.B, self.C = self.Am.array, self.Bm.array, self.Cm.array
        synth.fill(self.A, w.spec_a())
        synth.fill(self.B, w.spec_b())
        if nan_c:
            synth.fill_nan(self.C)
        else:
            synth.fill(self.C, w.spec_c())

    def free(self):
        for m in (self.Am, self.Bm, self.Cm):
            m.free()


def sample_rows(M, mb, count=16, seed=0):
    """Rows 0 and M-1, every block boundary -1/+0, and `count` random rows."""
    rows = {0, M - 1}
    for b in range(mb, M, mb):
        rows.update((b - 1, b))
    rng = np.random.default_rng(seed)
    rows.update(int(x) for x in rng.integers(0, M, count))
    return np.array(sorted(r for r in rows if 0 <= r < M), dtype=np.int64)


def reference_rows(w, A, B, rows):
    """Reference rows of the workload's product (initial C regenerated) and the
    gate denominator |alpha| (|A||B|)_ij + |beta| |C_in|_ij for those rows."""
    Cin = None
    if w.beta != 0.0:
        Cin = np.empty((len(rows), w.N))
        synth.fill_rows(Cin, rows, w.spec_c())
    ref, D = oracle.gemm_rows(w.alpha, A, B, w.beta, Cin, rows=rows)
    return ref, oracle.gate_denominator(w.alpha, D, w.beta, Cin)


def check_rows(w, pp, rows, gate=oracle.GATE):
    ref, D = reference_rows(w, pp.A, pp.B, rows)
    err = oracle.normalized_error(pp.C[rows], ref, D)
    assert err <= gate, f"normalised error {err:.3e} > {gate:.0e}"
    return err

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
    """Reference rows of the workload's product (initial C regenerated), the
    (|A||B|)_ij denominators of those rows and the initial C rows (None when
    beta == 0)."""
    Cin = None
    if w.beta != 0.0:
        Cin = np.empty((len(rows), w.N))
        synth.fill_rows(Cin, rows, w.spec_c())
    ref, D = oracle.gemm_rows(w.alpha, A, B, w.beta, Cin, rows=rows)
    return ref, D, Cin


def gate_errors(C, ref, alpha, D, beta, Cin, gate=oracle.GATE, label=""):
    """Both error figures of a result against the reference, printed:
    literal max |C - Cref| / (|A||B|)_ij and the generalised form with
    |alpha| (|A||B|)_ij + |beta| |C_in|_ij.  The literal metric is the gate
    wherever beta == 0; with beta != 0 the generalised one is (one rounding of
    alpha*S + beta*C can exceed 1e-12 of (|A||B|)_ij where |beta C_in| is much
    larger), and the literal figure is reported beside it."""
    lit, gen = oracle.errors(C, ref, alpha, D, beta, Cin)
    print(f"  {label}error literal {lit:.3e} generalised {gen:.3e}", flush=True)
    if beta == 0.0:
        assert lit <= gate, f"literal normalised error {lit:.3e} > {gate:.0e}"
    assert gen <= gate, f"generalised normalised error {gen:.3e} > {gate:.0e}"
    return lit, gen


def check_rows(w, pp, rows, gate=oracle.GATE, label=""):
    """Check the given rows of pp.C against the reference; returns the gated error."""
    ref, D, Cin = reference_rows(w, pp.A, pp.B, rows)
    lit, gen = gate_errors(pp.C[rows], ref, w.alpha, D, w.beta, Cin, gate, label=f"{label}{len(rows)} rows: ")
    return lit if w.beta == 0.0 else gen


class HipRuntime:
    """A few calls of the HIP runtime that the library itself links (the
    soname resolves to the copy already loaded with libooc).  torch carries a
    HIP runtime of its own; a second runtime in the process could not see the
    GPU after the library's had initialised it, so the GPU tests create their
    caller-owned streams here."""

    def __init__(self):
        import ctypes
        self._ct = ctypes
        self.lib = ctypes.CDLL("libamdhip64.so.7")
        self.lib.hipStreamCreateWithFlags.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint]
        self.lib.hipStreamDestroy.argtypes = [ctypes.c_void_p]
        self.lib.hipStreamSynchronize.argtypes = [ctypes.c_void_p]
        self.lib.hipMemGetInfo.argtypes = [ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
        self.lib.hipSetDevice.argtypes = [ctypes.c_int]
        self.lib.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
        self.lib.hipFree.argtypes = [ctypes.c_void_p]

    def _check(self, rc, what):
        if rc != 0:
            raise RuntimeError(f"{what} failed with HIP error {rc}")

    def set_device(self, dev):
        self._check(self.lib.hipSetDevice(dev), "hipSetDevice")

    def stream_create(self):
        """A non-blocking stream at the default priority."""
        s = self._ct.c_void_p()
        self._check(self.lib.hipStreamCreateWithFlags(self._ct.byref(s), 1), "hipStreamCreateWithFlags")
        return s.value

    def stream_destroy(self, s):
        self._check(self.lib.hipStreamDestroy(s), "hipStreamDestroy")

    def stream_synchronize(self, s):
        self._check(self.lib.hipStreamSynchronize(s), "hipStreamSynchronize")

    def device_synchronize(self):
        self._check(self.lib.hipDeviceSynchronize(), "hipDeviceSynchronize")

    def malloc(self, nbytes):
        p = self._ct.c_void_p()
        self._check(self.lib.hipMalloc(self._ct.byref(p), nbytes), "hipMalloc")
        return p.value

    def free(self, p):
        self._check(self.lib.hipFree(p), "hipFree")

    def mem_free(self):
        fr, tot = self._ct.c_size_t(), self._ct.c_size_t()
        self._check(self.lib.hipMemGetInfo(self._ct.byref(fr), self._ct.byref(tot)), "hipMemGetInfo")
        return fr.value

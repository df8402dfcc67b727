"""The allocation-free split-BF16 entry point (static device scratch) against
the allocating one, through the C ABI: bit-identical results on two calls in a
row, the second with a smaller input (the scratch keeps the first call's
contents), no change in free device memory, and sizes beyond the scratch
rejected before any device work."""
import numpy as np
import pytest

import synth
import paper_1808_05056_amd as ooc
from gpu_helpers import HipRuntime

pytestmark = pytest.mark.gpu

CALLS = [
    # m, n, k, s, alpha, beta, exponent spread
    (300, 260, 2048, 5, 1.0, 0.5, 10),
    (129, 77, 500, 6, -0.75, 0.0, 4),  # smaller: stale planes and sums of the first call stay in the scratch
]


def _operands(m, n, k, seed, spread):
    A = np.ascontiguousarray(synth.matrix(m, k, synth.spec(seed, 0, synth.NORMAL, row_exp=(-spread, spread))))
    B = np.ascontiguousarray(synth.matrix(k, n, synth.spec(seed, 1, synth.NORMAL, col_exp=(-spread, spread))))
    C = np.ascontiguousarray(synth.matrix(m, n, synth.spec(seed, 2, synth.UNIFORM)))
    return A, B, C


def test_noalloc_matches_allocating_entry_point_twice():
    hip = HipRuntime()
    hip.set_device(0)
    stream = hip.stream_create()
    try:
        for x, (m, n, k, s, alpha, beta, spread) in enumerate(CALLS):
            print(f"noalloc call {x}: m={m} n={n} k={k} s={s}", flush=True)
            A, B, C0 = _operands(m, n, k, 700 + x, spread)
            dA, dB = ooc.DeviceBuffer(A.nbytes), ooc.DeviceBuffer(B.nbytes)
            dC1, dC2 = ooc.DeviceBuffer(C0.nbytes), ooc.DeviceBuffer(C0.nbytes)
            dA.upload(A); dB.upload(B); dC1.upload(C0); dC2.upload(C0)
            ooc.ooc_split_gemm_device(m, n, k, s, alpha, dA.ptr, k, dB.ptr, n, beta, dC1.ptr, n)
            free0 = hip.mem_free()
            ooc.ooc_split_gemm_device_noalloc(m, n, k, s, alpha, dA.ptr, k, dB.ptr, n, beta, dC2.ptr, n,
                                              stream=stream)
            hip.stream_synchronize(stream)
            if x == 0:
                # the first call on the device loads the code object holding the
                # static scratch array (once per process): at most the array and
                # a little code, never per call
                assert free0 - hip.mem_free() <= ooc.NOALLOC_SCRATCH_BYTES + (8 << 20)
            else:
                assert hip.mem_free() == free0
            want, got = dC1.download((m, n)), dC2.download((m, n))
            assert np.all(np.isfinite(got))
            assert np.array_equal(got, want), np.max(np.abs(got - want))
            for b in (dA, dB, dC1, dC2):
                b.free()
    finally:
        hip.stream_destroy(stream)


def test_noalloc_rejects_workspace_beyond_scratch():
    # 4096 x 4096 x 8192 at s = 6 needs far more than the scratch: refused
    # before any device work (the pointers are never dereferenced)
    with pytest.raises(ooc.OOCError) as ei:
        ooc.ooc_split_gemm_device_noalloc(4096, 4096, 8192, 6, 1.0, 16, 8192, 16, 4096, 0.0, 16, 4096)
    assert ei.value.status == 8  # OOC_ERR_CAPACITY

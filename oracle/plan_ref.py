"""Reference for the paper's partitioner -- TEST INFRASTRUCTURE ONLY.

Section V: the partitioner splits A into h equal horizontal slices, B into w
equal vertical slices and C into h x w blocks, so that the data needed to
update any two C blocks of one column fits in the device memory dMemSize.
Those data are two C blocks, the two A slices they use and the one B slice of
their column:
    footprint(h, w) = 2*mb*K + K*nb + 2*mb*nb   elements,  mb = ceil(M/h), nb = ceil(N/w).
A plan with a single block (h = w = 1) needs no second buffer, so its
footprint is M*K + K*N + M*N; this is the in-core case (Section VI: the GPUs
with 12 GB switch to out-of-core above N = 22528, the 6 GB Xeon Phi above
N = 16384, which is exactly 24*N^2 <= memory).

Readings where the paper is silent (each listed in the design notes):
  * "equal slices" with a remainder: the last slice is the ragged remainder
    (mb = ceil(M/h)); h values that would leave an empty slice are skipped.
  * "fit": footprint <= budget (the 6 GiB threshold is met with equality).
  * among feasible (h, w): the smallest w, then the smallest h.  This is the
    only order consistent with the worked example (A 4x8, B 8x4, 44 elements
    gives h = 4, w = 2); minimising h*w instead would give h = 2, w = 4.
Sizes here are counted in elements (8 bytes each).
"""
import math


def _ceil(a, b):
    return -(-a // b)


def footprint(M, N, K, h, w):
    mb, nb = _ceil(M, h), _ceil(N, w)
    if h * w == 1:
        return M * K + K * N + M * N
    return 2 * mb * K + K * nb + 2 * mb * nb


def _proper(n, parts):
    """True if splitting n into `parts` slices of ceil(n/parts) leaves none empty."""
    return parts >= 1 and _ceil(n, _ceil(n, parts)) == parts


def feasible(M, N, K, h, w, budget_elems):
    return footprint(M, N, K, h, w) <= budget_elems


def partition(M, N, K, budget_elems):
    """(h, w) of the paper's partitioner, or None if no split fits.

    For each w = 1, 2, ... the footprint depends on h only through
    mb = ceil(M/h) and does not grow as h grows (h >= 2), so the smallest
    feasible h is found by bisection; it is always a proper split.
    """
    for w in range(1, N + 1):
        if not _proper(N, w):
            continue
        if feasible(M, N, K, 1, w, budget_elems):
            return (1, w)
        if M == 1 or not feasible(M, N, K, M, w, budget_elems):
            continue
        lo, hi = 1, M  # lo infeasible, hi feasible
        while hi - lo > 1:
            mid = (lo + hi) // 2
            if feasible(M, N, K, mid, w, budget_elems):
                hi = mid
            else:
                lo = mid
        return (hi, w)
    return None


def partition_bruteforce(M, N, K, budget_elems):
    """All-pairs scan of the same rule, for small problems."""
    best = None
    for w in range(1, N + 1):
        if not _proper(N, w):
            continue
        for h in range(1, M + 1):
            if not _proper(M, h):
                continue
            if feasible(M, N, K, h, w, budget_elems):
                cand = (w, h)
                if best is None or cand < best:
                    best = cand
    return None if best is None else (best[1], best[0])


def max_incore_square(mem_bytes, step=1024):
    """Largest N (multiple of `step`) whose square product is in-core (h = w = 1)."""
    n = step
    while footprint(n + step, n + step, n + step, 1, 1) * 8 <= mem_bytes:
        n += step
    return n if footprint(n, n, n, 1, 1) * 8 <= mem_bytes else 0

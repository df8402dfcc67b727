"""Reference for the pipeline's ordering -- TEST INFRASTRUCTURE ONLY.

The paper's MMOOC (Section V, Fig. 2 and Fig. 4) runs five stages per C block
c_ij: S(b_j) sends a B slice, S(a_i) an A slice, S(c_ij) a C block, DGEMM
updates c_ij, R(c_ij) returns it.  Events order them so that no device buffer
is overwritten while an operation still reads it.  The events are
  rA[idx]  A slice of block idx has arrived     rB[j]   B slice of column j has arrived
  rC[idx]  C block idx has arrived              eA[idx] the DGEMM of block idx is done
  eC[idx]  C block idx is back on the host
with blocks numbered idx = i + j*h (column by column).  A and C slices are
double-buffered by the parity of idx, the B slice is single-buffered.

This module holds
  * paper_rules(h, w, beta_nonzero): the ordering those events impose, as
    (later, earlier) pairs of logical operations, for checking that a schedule
    in the paper's configuration implies every one of them;
  * happens_before / check_hazards / check_cover: generic checks of an
    operation list (stream order + explicit waits);
  * execute: runs an operation list on the CPU, in a random order that
    respects stream order and waits, with numpy copies into a simulated device
    arena, so a missing wait shows up as a wrong result.

An operation is a dict with keys
  kind 'h2d' | 'd2h' | 'gemm' | other kernels ('exp', 'slice', 'split_gemm', 'scale')
  stream, waits (list of earlier op indices), task
  copies: mat ('A'|'B'|'C'), row0, col0, rows, cols, dev_off, dev_ld (elements)
  gemm:   m, n, k, i0, j0, k0, off_a, lda, off_b, ldb, off_c, ldc, alpha, beta
          and optionally off_d, ldd, gamma: c = alpha*a@b + beta*c + gamma*d;
          transb: b is stored transposed (n x k); lower: only the elements of
          c with i0 + r >= j0 + c (on or below the diagonal of the whole
          result) are computed and written
  other kernels: reads / writes, lists of (offset, rows, cols, ld) device regions.
"""
import random

import numpy as np

# logical operation names used by paper_rules
H2D_A, H2D_B, H2D_C, GEMM, D2H_C = "S(a)", "S(b)", "S(c)", "DGEMM", "R(c)"


def paper_rules(h, w, beta_nonzero=True):
    """Ordering imposed by the events of the paper's MMOOC for an h x w split.

    Returns a list of ((name, index), (name, index)) = (later, earlier): the
    later operation may start only after the earlier one completed.  Indices
    are block numbers idx (or the column j for S(b)).  Where a rule would
    refer to block -1 it is dropped (the listing's wait on eA[idx-1] at the
    first block is read as guarded by idx > 0).
    """
    rules = []
    n = h * w
    for idx in range(n):
        i, j = idx % h, idx // h
        # the DGEMM of block idx waits for rA[idx], rB[j], rC[idx]
        rules.append(((GEMM, idx), (H2D_A, idx)))
        rules.append(((GEMM, idx), (H2D_B, j)))
        if beta_nonzero:
            rules.append(((GEMM, idx), (H2D_C, idx)))
        # block idx returns after its DGEMM
        rules.append(((D2H_C, idx), (GEMM, idx)))
        if idx + 1 < n and idx >= 1:
            # the A slice of block idx+1 reuses the buffer of block idx-1 (parity)
            rules.append(((H2D_A, idx + 1), (GEMM, idx - 1)))
            # the C block idx+1 reuses the buffer of block idx-1 once it is home
            if beta_nonzero:
                rules.append(((H2D_C, idx + 1), (D2H_C, idx - 1)))
        if i == h - 1 and j + 1 < w:
            # the single B buffer is refilled after the column's last DGEMMs
            rules.append(((H2D_B, j + 1), (GEMM, idx)))
            if idx >= 1:
                rules.append(((H2D_B, j + 1), (GEMM, idx - 1)))
    return rules


def logical_names(ops, h):
    """Map logical (name, index) -> op index for a schedule of the paper's
    configuration (K not split; tasks numbered idx = i + j*h)."""
    out = {}
    for x, op in enumerate(ops):
        t = op["task"]
        if op["kind"] == "gemm":
            out[(GEMM, t)] = x
        elif op["kind"] == "d2h":
            out[(D2H_C, t)] = x
        elif op["kind"] == "h2d":
            if op["mat"] == "A":
                out[(H2D_A, t)] = x
            elif op["mat"] == "C":
                out[(H2D_C, t)] = x
            elif op["mat"] == "B":
                out[(H2D_B, t // h)] = x
    return out


def predecessors(ops):
    """Direct predecessors of each op: the previous op on its stream plus its waits."""
    last = {}
    preds = []
    for x, op in enumerate(ops):
        p = set(op.get("waits", ()))
        for y in p:
            if not (0 <= y < x):
                raise ValueError(f"op {x} waits on op {y}, which is not earlier in the list")
        s = op["stream"]
        if s in last:
            p.add(last[s])
        last[s] = x
        preds.append(sorted(p))
    return preds


def happens_before(ops):
    """reach[x] = bitmask of ops that complete before op x starts."""
    preds = predecessors(ops)
    reach = []
    for x in range(len(ops)):
        m = 0
        for y in preds[x]:
            m |= reach[y] | (1 << y)
        reach.append(m)
    return reach


def _regions(op):
    """(reads, writes) as lists of (first_elem, rows, cols, ld) in the device arena."""
    k = op["kind"]
    if k == "h2d":
        return [], [(op["dev_off"], op["rows"], op["cols"], op["dev_ld"])]
    if k == "d2h":
        return [(op["dev_off"], op["rows"], op["cols"], op["dev_ld"])], []
    if k in ("gemm", "split_gemm"):
        b = (op["off_b"], op["n"], op["k"], op["ldb"]) if op.get("transb") else (op["off_b"], op["k"], op["n"], op["ldb"])
        reads = [(op["off_a"], op["m"], op["k"], op["lda"]), b]
        if k == "split_gemm" and op.get("len_w", 0) > 0:
            ws = (op["off_w"], 1, op["len_w"], op["len_w"])
            if op["beta"] != 0.0:
                reads.append((op["off_c"], op["m"], op["n"], op["ldc"]))
            if op.get("gamma", 0.0) != 0.0:
                reads.append((op["off_d"], op["m"], op["n"], op["ldd"]))
            return reads + [ws], [(op["off_c"], op["m"], op["n"], op["ldc"]), ws]
        if op["beta"] != 0.0:
            reads.append((op["off_c"], op["m"], op["n"], op["ldc"]))
        if op.get("gamma", 0.0) != 0.0:
            reads.append((op["off_d"], op["m"], op["n"], op["ldd"]))
        return reads, [(op["off_c"], op["m"], op["n"], op["ldc"])]
    return list(op.get("reads", [])), list(op.get("writes", []))


def _span(r):
    off, rows, cols, ld = r
    if rows == 0 or cols == 0:
        return None
    return (off, off + (rows - 1) * ld + cols)


def _overlap(r1, r2):
    """Exact test whether two strided 2-D regions share an element."""
    s1, s2 = _span(r1), _span(r2)
    if s1 is None or s2 is None or s1[1] <= s2[0] or s2[1] <= s1[0]:
        return False
    o1, n1, c1, l1 = r1
    o2, n2, c2, l2 = r2
    a = np.zeros(max(s1[1], s2[1]) - min(s1[0], s2[0]), dtype=np.uint8)
    base = min(s1[0], s2[0])
    for (o, n, c, l), bit in ((r1, 1), (r2, 2)):
        for r in range(n):
            a[o - base + r * l: o - base + r * l + c] |= bit
    return bool(np.any(a == 3))


def check_hazards(ops):
    """List of (x, y) pairs of unordered ops that touch a common device
    element with at least one of them writing it (empty list = race free)."""
    reach = happens_before(ops)
    rw = [_regions(op) for op in ops]
    bad = []
    for x in range(len(ops)):
        rx, wx = rw[x]
        for y in range(x):
            if (reach[x] >> y) & 1:
                continue
            ry, wy = rw[y]
            conflict = any(_overlap(a, b) for a in wx for b in ry + wy) or any(_overlap(a, b) for a in rx for b in wy)
            if conflict:
                bad.append((x, y))
    return bad


def _cells(ops, M, N):
    """Row and column boundaries of every rectangle the ops touch in C: the
    grid they form has cells that each op covers entirely or not at all."""
    rb, cb = {0, M}, {0, N}
    for op in ops:
        if op["kind"] == "d2h" or op["kind"] in ("gemm", "split_gemm"):
            r0, c0, r, c = _host_rect(op)
            rb.update((r0, r0 + r))
            cb.update((c0, c0 + c))
    return sorted(x for x in rb if 0 <= x <= M), sorted(x for x in cb if 0 <= x <= N)


def _host_rect(op):
    """(row0, col0, rows, cols) of C that an op returns (d2h) or updates (GEMM)."""
    if op["kind"] == "d2h":
        return op["row0"], op["col0"], op["rows"], op["cols"]
    return op["i0"], op["j0"], op["m"], op["n"]


def check_cover(ops, M, N, K, returns_home=True, lower=False):
    """Coverage of the result by an operation list.  Returns a list of
    problems (empty = fine); with lower, only the elements C_ij with i >= j
    are owed (cells wholly above the diagonal are not checked):
      * every C element is returned to the host (d2h of mat 'C') exactly once
        (with returns_home=False, for C that stays on the device between the
        steps of an accumulation session: never);
      * for every C element, the K ranges [k0, k0 + k) of the GEMM ops that
        update it tile [0, K) exactly: no gap, no overlap, no repeat (so every
        product term A_ik B_kj is added exactly once); with K == 0 every GEMM
        op of the element has k == 0;
      * the element's d2h is ordered after every GEMM op that updates it
        (stream order and waits), so the host receives the finished value.
    """
    problems = []
    rows, cols = _cells(ops, M, N)
    reach = happens_before(ops)
    gemms = [x for x, op in enumerate(ops) if op["kind"] in ("gemm", "split_gemm")]
    homes = [x for x, op in enumerate(ops) if op["kind"] == "d2h" and op.get("mat", "C") == "C"]

    def covers(op, r0, c0):
        a, b, r, c = _host_rect(op)
        return a <= r0 < a + r and b <= c0 < b + c

    for ri in range(len(rows) - 1):
        for ci in range(len(cols) - 1):
            r0, c0 = rows[ri], cols[ci]
            if rows[ri + 1] <= r0 or cols[ci + 1] <= c0:
                continue
            cell = f"C[{r0}:{rows[ri + 1]}, {c0}:{cols[ci + 1]}]"
            if lower and rows[ri + 1] - 1 < c0:
                continue  # every element of the cell lies above the diagonal
            home = [x for x in homes if covers(ops[x], r0, c0)]
            if len(home) != (1 if returns_home else 0):
                problems.append(f"{cell} returned {len(home)} times")
            ivs = sorted((ops[x]["k0"], ops[x]["k"], x) for x in gemms if covers(ops[x], r0, c0))
            if K > 0:
                at = 0
                for k0, k, x in ivs:
                    if k0 > at:
                        problems.append(f"{cell}: k range [{at}, {k0}) not computed")
                    elif k0 < at:
                        problems.append(f"{cell}: k range [{k0}, {min(at, k0 + k)}) computed twice (op {x})")
                    at = max(at, k0 + k)
                if at < K:
                    problems.append(f"{cell}: k range [{at}, {K}) not computed")
                elif at > K:
                    problems.append(f"{cell}: k range reaches {at} > K = {K}")
            elif any(k != 0 for _, k, _ in ivs):
                problems.append(f"{cell}: K = 0 but a GEMM op has k > 0")
            for h in home:
                for _, _, x in ivs:
                    if not (reach[h] >> x) & 1:
                        problems.append(f"{cell}: d2h op {h} is not ordered after GEMM op {x}")
    return problems


def execute(ops, A, B, C, arena_elems, seed=0, poison=np.nan, kernels=None, arena=None):
    """Run the operation list on the CPU.

    Ops are taken in a random order that respects stream order and waits.  The
    device arena starts filled with `poison`, unless an existing arena (a
    float64 array of at least arena_elems entries) is passed, which is then
    used and updated in place (device memory that outlives one operation
    list, as in an accumulation session).  GEMM ops compute
    alpha*a@b + beta*c on the arena views (beta == 0: c is not read).  Other
    kernel kinds are run by kernels[kind](op, arena) when given.
    C (host) is updated in place by the d2h ops.
    """
    if arena is None:
        arena = np.full(arena_elems, poison, dtype=np.float64)
    elif arena.shape[0] < arena_elems:
        raise ValueError("arena smaller than the operation list needs")
    host = {"A": A, "B": B, "C": C}
    preds = predecessors(ops)
    n = len(ops)
    done = [False] * n
    rng = random.Random(seed)
    ready = [x for x in range(n) if not preds[x]]
    remaining = {x: len(preds[x]) for x in range(n)}
    succ = [[] for _ in range(n)]
    for x in range(n):
        for y in preds[x]:
            succ[y].append(x)

    def view(off, rows, cols, ld):
        if rows == 0 or cols == 0:
            return np.zeros((rows, cols))
        return np.lib.stride_tricks.as_strided(arena[off:], shape=(rows, cols), strides=(ld * 8, 8))

    while ready:
        x = ready.pop(rng.randrange(len(ready)))
        op = ops[x]
        k = op["kind"]
        if k == "h2d":
            src = host[op["mat"]][op["row0"]:op["row0"] + op["rows"], op["col0"]:op["col0"] + op["cols"]]
            view(op["dev_off"], op["rows"], op["cols"], op["dev_ld"])[...] = src
        elif k == "d2h":
            host[op["mat"]][op["row0"]:op["row0"] + op["rows"], op["col0"]:op["col0"] + op["cols"]] = \
                view(op["dev_off"], op["rows"], op["cols"], op["dev_ld"])
        elif k == "gemm":
            a = view(op["off_a"], op["m"], op["k"], op["lda"])
            if op.get("transb"):
                b = view(op["off_b"], op["n"], op["k"], op["ldb"]).T
            else:
                b = view(op["off_b"], op["k"], op["n"], op["ldb"])
            c = view(op["off_c"], op["m"], op["n"], op["ldc"])
            prod = a @ b if op["k"] else np.zeros((op["m"], op["n"]))
            if op["alpha"] == 0.0:
                prod = np.zeros_like(prod)
            res = op["alpha"] * prod
            if op["beta"] != 0.0:
                res = res + op["beta"] * c
            if op.get("gamma", 0.0) != 0.0:
                res = res + op["gamma"] * view(op["off_d"], op["m"], op["n"], op["ldd"])
            if op.get("lower"):
                r, cc = np.indices((op["m"], op["n"]))
                keep = op["i0"] + r >= op["j0"] + cc
                c[keep] = res[keep]
            else:
                c[...] = res
        else:
            if kernels is None or k not in kernels:
                raise ValueError(f"no CPU model for op kind {k}")
            kernels[k](op, arena)
        done[x] = True
        for y in succ[x]:
            remaining[y] -= 1
            if remaining[y] == 0:
                ready.append(y)
    if not all(done):
        raise RuntimeError("operation list has a cycle or an unsatisfiable wait")
    return C

"""The synthetic workloads: shapes, seeds, value distributions, alpha/beta and budgets.

Each workload is the paper's problem (C = alpha*A*B + beta*C in FP64, row-major,
operands in host memory, device memory capped by a budget) at a stated size.
The paper measures square products with unstated matrix values (Section VI);
these seeded synthetic matrices stand in for them.
"""
import math
from dataclasses import dataclass, field

from . import UNIFORM, NORMAL, MAT_A, MAT_B, MAT_C, spec, lib

KiB, MiB, GiB = 1 << 10, 1 << 20, 1 << 30


@dataclass
class Workload:
    name: str
    M: int
    N: int
    K: int
    alpha: float
    beta: float
    budget: int
    seed: int
    dist_a: int = UNIFORM
    dist_b: int = UNIFORM
    dist_c: int = UNIFORM
    a_row_exp: tuple = (0.0, 0.0)
    b_col_exp: tuple = (0.0, 0.0)
    note: str = ""
    extra: dict = field(default_factory=dict)

    def spec_a(self):
        return spec(self.seed, MAT_A, self.dist_a, row_exp=self.a_row_exp)

    def spec_b(self):
        return spec(self.seed, MAT_B, self.dist_b, col_exp=self.b_col_exp)

    def spec_c(self):
        return spec(self.seed, MAT_C, self.dist_c)

    @property
    def flops(self):
        return 2.0 * self.M * self.N * self.K

    def host_bytes(self):
        return 8 * (self.M * self.K + self.K * self.N + self.M * self.N)


SMALL = Workload("square-1024-budget-8MiB", 1024, 1024, 1024, 1.0, 0.0, 8 * MiB, seed=1,
                 note="24 MiB problem tiled through an 8 MiB device budget")
SQUARE = Workload("square-32768-budget-4GiB", 32768, 32768, 32768, 1.5, 0.5, 4 * GiB, seed=2,
                  dist_c=UNIFORM, note="8 GiB per matrix, 4 GiB device budget")
SCALED = Workload("scaled-65536x16384x32768-budget-8GiB", 65536, 16384, 32768, 1.0, 0.0, 8 * GiB, seed=3,
                  dist_a=NORMAL, dist_b=NORMAL, a_row_exp=(-20.0, 20.0), b_col_exp=(-20.0, 20.0),
                  note="normal entries, rows of A and columns of B scaled by 2^U(-20,20)")
TALL = Workload("tall-262144x8192x8192-budget-2GiB", 262144, 8192, 8192, 1.0, 1.0, 2 * GiB, seed=5,
                note="A is 16 GiB; C read and written (beta=1)")

BY_NAME = {w.name: w for w in (SMALL, SQUARE, SCALED, TALL)}

_PROBLEM_MAT = 6  # generator matrix id reserved for drawing problem shapes


def _u01(seed, r, c):
    """A uniform [0,1) draw from the counter-based generator."""
    v = lib().syn_entry(spec(seed, _PROBLEM_MAT, UNIFORM), r, c)
    return (v + 1.0) / 2.0


def problem_batch(seed, count=64, lo=4096, hi=24576, budget_lo=256 * MiB, budget_hi=8 * GiB):
    """Problems with M, N, K log-uniform in [lo, hi] and budgets log-uniform in
    [budget_lo, budget_hi] rounded down to 2 MiB; entries uniform[-1, 1].

    seed 4 is the evaluation batch and seed 40 the disjoint training batch.
    """
    out = []
    for p in range(count):
        dims = [int(round(math.exp(math.log(lo) + (math.log(hi) - math.log(lo)) * _u01(seed, p, q))))
                for q in range(3)]
        b = math.exp(math.log(budget_lo) + (math.log(budget_hi) - math.log(budget_lo)) * _u01(seed, p, 3))
        budget = max(2 * MiB, int(b) // (2 * MiB) * (2 * MiB))
        out.append(Workload(f"batch{seed}-{p}", dims[0], dims[1], dims[2], 1.0, 0.0, budget,
                            seed=seed * 1000 + p))
    return out


def tall_batch(seed, count=8, m_lo=65536, m_hi=262144, lo=4096, hi=8192, budget_lo=1 * GiB, budget_hi=4 * GiB):
    """Tall problems: M log-uniform in [m_lo, m_hi], N and K log-uniform in
    [lo, hi], budgets log-uniform in [budget_lo, budget_hi] rounded down to
    2 MiB, beta = 1 for odd-numbered problems (0 otherwise); entries
    uniform[-1, 1].  seed 41 widens the planner's training batch to the shapes
    of the tall workload."""
    out = []
    for p in range(count):
        m = int(round(math.exp(math.log(m_lo) + (math.log(m_hi) - math.log(m_lo)) * _u01(seed, p, 0))))
        n, k = (int(round(math.exp(math.log(lo) + (math.log(hi) - math.log(lo)) * _u01(seed, p, q))))
                for q in (1, 2))
        b = math.exp(math.log(budget_lo) + (math.log(budget_hi) - math.log(budget_lo)) * _u01(seed, p, 3))
        budget = max(2 * MiB, int(b) // (2 * MiB) * (2 * MiB))
        out.append(Workload(f"tall{seed}-{p}", m, n, k, 1.0, float(p % 2), budget, seed=seed * 1000 + p))
    return out

// Planning: arena layout, the paper's partitioner, candidate plans and the
// analytic cost model (a discrete-event simulation of the operation list).
#include <algorithm>
#include <cmath>
#include <limits>
#include <map>
#include <mutex>
#include <set>
#include <thread>
#include <tuple>

#include "internal.hpp"
#include "kernels.hpp"

namespace ooc {

const Machine& machine() {
  static Machine m;
  return m;
}

int64_t split_workspace_elems(const Problem& pb, const ooc_plan_t& plan) {
  if (plan.precision == OOC_FP64 || pb.keff() == 0) return 0;
  // slice planes of one A panel and one B panel plus their exponents and the slice-sum tile
  return ceil_div((int64_t)split_workspace_bytes(plan.mb, plan.nb, plan.kb, plan.slices, slice_format(plan.precision)),
                  8);
}

ooc_status plan_layout(const Problem& pb, const ooc_plan_t& plan, Layout* lay) {
  const int64_t K = pb.keff();
  if (plan.mb <= 0 || plan.nb <= 0) return fail(OOC_ERR_ARG, "plan: mb and nb must be positive");
  if (K > 0 && plan.kb <= 0) return fail(OOC_ERR_ARG, "plan: kb must be positive");
  if (plan.nstreams < 1 || plan.nstreams > 3) return fail(OOC_ERR_ARG, "plan: nstreams must be 1, 2 or 3");
  if (plan.order < 0 || plan.order > 5) return fail(OOC_ERR_ARG, "plan: unknown order");
  if (plan.nbuf_c < 1 || (K > 0 && (plan.nbuf_a < 1 || plan.nbuf_b < 1)))
    return fail(OOC_ERR_ARG, "plan: every operand needs at least one buffer");
  if (plan.precision != OOC_FP64 && plan.precision != OOC_SPLIT_BF16 && plan.precision != OOC_SPLIT_INT8)
    return fail(OOC_ERR_ARG, "plan: unknown precision");
  if (plan.precision != OOC_FP64 && (plan.slices < 1 || plan.slices > 8))
    return fail(OOC_ERR_ARG, "plan: slices must be 1..8");
  if (plan.nbuf_d < 0) return fail(OOC_ERR_ARG, "plan: nbuf_d must be >= 0");
  if (plan.group < 0) return fail(OOC_ERR_ARG, "plan: group must be >= 0");
  if (pb.lower && plan.precision != OOC_FP64)
    return fail(OOC_ERR_ARG, "plan: lower-triangle products run in FP64 precision only");
  // clamp to the problem (a block larger than the matrix is the matrix)
  const int64_t mb = std::min(plan.mb, std::max<int64_t>(pb.M, 1));
  const int64_t nb = std::min(plan.nb, std::max<int64_t>(pb.N, 1));
  const int64_t kb = K > 0 ? std::min(plan.kb, K) : 0;
  const int64_t h = ceil_div(pb.M, mb), w = ceil_div(pb.N, nb);
  Layout L;
  const bool single = (h * w == 1) && (K == 0 || kb >= K);
  // resident C (accumulation sessions) needs no C buffers
  const int64_t slot_c = pb.c_resident ? 0 : mb * nb;
  if (pb.base < 0 || (pb.c_resident && (pb.c_ld < pb.N || pb.base < (pb.M - 1) * pb.c_ld + pb.N)))
    return fail(OOC_ERR_ARG, "plan: resident C region malformed");
  if (single) {
    // one block: each operand needs exactly one buffer (the in-core case)
    L.slotA = mb * kb;
    L.slotB = kb * nb;
    L.slotC = slot_c;
    L.offA = pb.base;
    L.offB = L.offA + (K > 0 ? L.slotA : 0);
    L.offC = L.offB + (K > 0 ? L.slotB : 0);
    L.offD = L.offC + L.slotC;
    L.offW = L.offD;
  } else {
    L.slotA = mb * kb;
    L.slotB = kb * nb;
    L.slotC = slot_c;
    L.offA = pb.base;
    L.offB = L.offA + (K > 0 ? plan.nbuf_a * L.slotA : 0);
    L.offC = L.offB + (K > 0 ? plan.nbuf_b * L.slotB : 0);
    L.offD = L.offC + plan.nbuf_c * L.slotC;
    // staging buffers for the initial C (only when C is read at all; not for
    // lower-triangle products, whose straddling blocks carry their upper part
    // through their own buffer)
    if (plan.nbuf_d > 0 && pb.beta != 0.0 && !pb.c_resident && !pb.lower) {
      L.nbufD = plan.nbuf_d;
      L.slotD = mb * nb;
    }
    L.offW = L.offD + (int64_t)L.nbufD * L.slotD;
  }
  ooc_plan_t p2 = plan;
  p2.mb = mb; p2.nb = nb; p2.kb = kb;
  L.lenW = split_workspace_elems(pb, p2);
  if (L.lenW > 0) L.offW = ceil_div(L.offW, 32) * 32;  // 256-byte aligned workspace
  L.bytes = (uint64_t)(L.offW + L.lenW) * 8u;
  *lay = L;
  return OOC_OK;
}

// ---- the paper's partitioner -----------------------------------------------------

static inline uint64_t paper_footprint(int64_t M, int64_t N, int64_t K, int64_t h, int64_t w) {
  const int64_t mb = ceil_div(M, h), nb = ceil_div(N, w);
  if (h * w == 1) return (uint64_t)(M * K + K * N + M * N);
  return (uint64_t)(2 * mb * K + K * nb + 2 * mb * nb);
}

static inline bool proper_split(int64_t n, int64_t parts) { return ceil_div(n, ceil_div(n, parts)) == parts; }

bool paper_partition(int64_t M, int64_t N, int64_t K, uint64_t budget_elems, int64_t* h_out, int64_t* w_out) {
  // Fewest vertical B slices w, then fewest horizontal A slices h, such that
  // two C blocks of one column, their two A slices and the column's B slice fit.
  for (int64_t w = 1; w <= N; ++w) {
    if (!proper_split(N, w)) continue;
    if (paper_footprint(M, N, K, 1, w) <= budget_elems) {
      *h_out = 1; *w_out = w;
      return true;
    }
    if (M == 1 || paper_footprint(M, N, K, M, w) > budget_elems) continue;
    int64_t lo = 1, hi = M;  // footprint(lo) > budget >= footprint(hi)
    while (hi - lo > 1) {
      int64_t mid = lo + (hi - lo) / 2;
      if (paper_footprint(M, N, K, mid, w) <= budget_elems) hi = mid; else lo = mid;
    }
    *h_out = hi; *w_out = w;
    return true;
  }
  return false;
}

bool paper_plan(const Problem& pb, uint64_t budget_bytes, ooc_plan_t* plan, int precision, int slices) {
  // The paper's rule (fewest w, then fewest h) over the plan's full device
  // layout; for FP64 the layout is exactly the partitioner's footprint, for
  // split-BF16 it adds the slice workspace, which also shrinks as h grows.
  const int64_t K = pb.keff();
  auto make = [&](int64_t h, int64_t w) {
    ooc_plan_t p{};
    p.mb = ceil_div(pb.M, h);
    p.nb = ceil_div(pb.N, w);
    p.kb = K;
    p.order = OOC_ORDER_COLS;
    p.nbuf_a = 2;
    p.nbuf_b = 1;
    p.nbuf_c = 2;
    p.nstreams = 2;
    p.precision = precision;
    p.slices = precision != OOC_FP64 ? slices : 0;
    p.nbuf_d = 0;
    return p;
  };
  auto fits = [&](int64_t h, int64_t w) {
    Layout lay;
    if (plan_layout(pb, make(h, w), &lay) != OOC_OK) return false;
    return lay.bytes <= budget_bytes;
  };
  if (precision == OOC_FP64) {
    int64_t h = 1, w = 1;
    if (!paper_partition(pb.M, pb.N, K, budget_bytes / 8, &h, &w)) return false;
    *plan = make(h, w);
    return true;
  }
  for (int64_t w = 1; w <= pb.N; ++w) {
    if (!proper_split(pb.N, w)) continue;
    if (fits(1, w)) { *plan = make(1, w); return true; }
    if (pb.M == 1 || !fits(pb.M, w)) continue;
    int64_t lo = 1, hi = pb.M;
    while (hi - lo > 1) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (fits(mid, w)) hi = mid; else lo = mid;
    }
    *plan = make(hi, w);
    return true;
  }
  return false;
}

// ---- cost model --------------------------------------------------------------------

static double kernel_seconds(const Machine& mc, int64_t m, int64_t n, int64_t k, int precision, int slices,
                             int32_t flags = 0) {
  if (m <= 0 || n <= 0) return mc.kernel_launch_s;
  const double tiles = (double)ceil_div(m, 128) * (double)ceil_div(n, 128);
  if (k <= 0) return mc.kernel_launch_s + (double)m * n * 16.0 / 4e12;
  // every 128 x 128 tile costs the same; a CU runs two at a time (one if
  // there are fewer tiles than CUs); a partial last wave of at most one tile
  // per CU runs at the one-workgroup rate
  const double tile_flops = 2.0 * 128.0 * 128.0 * (double)k * (1.0 + mc.kernel_k0 / (double)k);
  const double r2 = mc.kernel_tflops * 1e12 / mc.cus;      // per CU, two tiles in flight
  const double r1 = mc.kernel_tflops_1wg * 1e12 / mc.cus;  // per CU, one tile
  double t;
  if (tiles <= mc.cus) {
    t = tile_flops / r1;
  } else {
    const double per_wave = 2.0 * mc.cus;
    const double full = std::floor(tiles / per_wave);
    const double rest = tiles - full * per_wave;
    t = full * 2.0 * tile_flops / r2;
    if (rest > mc.cus) t += 2.0 * tile_flops / r2;
    else if (rest > 0) t += tile_flops / r1;
  }
  if ((k & 1) || (n & 1)) t *= mc.kernel_scalar_factor;
  if (precision != OOC_FP64) {
    // the slice-product kernels compute whole 256-row tiles of 128 columns
    // (BF16, INT8) or 256 (INT8, when their waves end sooner), one per CU at
    // a time, in waves of one tile per CU; every weight's pass over a tile
    // pays a pipeline start of split_k0 k of BF16 work (twice as many k at
    // the INT8 rate, which is about twice the BF16 one)
    const bool i8 = precision == OOC_SPLIT_INT8;
    const bool wide = i8 && split_i8_wide(m, n, mc.cus);
    const double tbn = wide ? 256.0 : 128.0;
    const double mp = std::ceil(m / 256.0) * 256.0, np = std::ceil(n / tbn) * tbn;
    const double products = slices * (slices + 1) / 2.0;
    const double stiles = (mp / 256.0) * (np / tbn);
    const double stile = 2.0 * 256.0 * tbn * (products * (double)k + (i8 ? 2.0 : 1.0) * slices * mc.split_k0);
    const double rate = !i8 ? mc.split_tflops_per_product
                            : (wide ? mc.int8_wide_tops_per_product : mc.int8_tops_per_product);
    const double ts = std::ceil(stiles / mc.cus) * stile / (rate * 1e12 / mc.cus);
    // slicing reads a panel and writes its planes; a panel whose slices the
    // previous product left in the workspace is not sliced again
    const double sliced = ((flags & OOC_OPF_REUSE_A) ? 0.0 : mp) + ((flags & OOC_OPF_REUSE_B) ? 0.0 : np);
    const double slice_s = sliced * k * (8.0 + (double)slice_format(precision) * slices) / 4e12;
    // the FP64 slice-sum tile is read and written once per weight (s weights)
    const double sum_s = (double)slices * 16.0 * mp * np / mc.hbm_bytes_per_s;
    return mc.kernel_launch_s * 6 + slice_s + sum_s + ts;
  }
  return mc.kernel_launch_s + t;
}

double simulate(const Problem& pb, const ooc_plan_t& plan, const std::vector<ooc_op>& ops,
                std::vector<double>* times) {
  // Event-driven fluid simulation: copies in one direction share that
  // direction's bandwidth, which drops to the duplex figure while the other
  // direction is busy; kernels share the device equally.
  const Machine& mc = machine();
  const size_t n = ops.size();
  if (n == 0) return 0.0;
  std::vector<double> work(n), done_at(n, -1.0);
  std::vector<int> cls(n);  // 0 H2D, 1 D2H, 2 kernel
  for (size_t x = 0; x < n; ++x) {
    const ooc_op& o = ops[x];
    if (o.kind == OOC_OP_H2D) { cls[x] = 0; work[x] = (double)o.rows * o.cols * 8.0; }
    else if (o.kind == OOC_OP_D2H) { cls[x] = 1; work[x] = (double)o.rows * o.cols * 8.0; }
    else {
      cls[x] = 2;
      work[x] = kernel_seconds(mc, o.rows, o.cols, o.k, o.kind == OOC_OP_SPLIT_GEMM ? plan.precision : OOC_FP64,
                               plan.slices, o.flags);
    }
  }
  const int ns = plan.nstreams;
  std::vector<std::vector<int>> q(ns);
  for (size_t x = 0; x < n; ++x) q[ops[x].stream].push_back((int)x);
  std::vector<size_t> head(ns, 0);
  std::vector<double> remaining(work);
  std::vector<double> lat(n, 0.0);  // latency left before a copy streams
  for (size_t x = 0; x < n; ++x) lat[x] = cls[x] < 2 ? mc.copy_latency_s : 0.0;
  std::vector<int> running;
  double now = 0.0;
  size_t completed = 0;
  auto ready = [&](int x) {
    const ooc_op& o = ops[x];
    for (int k = 0; k < o.nwait; ++k)
      if (done_at[o.wait[k]] < 0) return false;
    return true;
  };
  std::vector<char> active(ns, 0);
  if (times) times->assign(2 * n, 0.0);
  while (completed < n) {
    for (int s = 0; s < ns; ++s) {
      if (active[s] || head[s] >= q[s].size()) continue;
      int x = q[s][head[s]];
      if (ready(x)) {
        running.push_back(x);
        active[s] = 1;
        if (times) (*times)[2 * x] = now;
      }
    }
    if (running.empty()) return std::numeric_limits<double>::infinity();  // deadlock
    int nh = 0, nd = 0, nk = 0;
    for (int x : running) { if (lat[x] > 0) continue; if (cls[x] == 0) ++nh; else if (cls[x] == 1) ++nd; else ++nk; }
    const double bw_h = (nd ? mc.duplex_h2d_gbs : mc.h2d_gbs) * 1e9;
    const double bw_d = (nh ? mc.duplex_d2h_gbs : mc.d2h_gbs) * 1e9;
    double dt = std::numeric_limits<double>::infinity();
    std::vector<double> rate(running.size());
    for (size_t r = 0; r < running.size(); ++r) {
      int x = running[r];
      if (lat[x] > 0) { rate[r] = 0; dt = std::min(dt, lat[x]); continue; }
      if (cls[x] == 0) rate[r] = bw_h / nh;
      else if (cls[x] == 1) rate[r] = bw_d / nd;
      else rate[r] = 1.0 / nk;
      dt = std::min(dt, remaining[x] / rate[r]);
    }
    now += dt;
    std::vector<int> still;
    for (size_t r = 0; r < running.size(); ++r) {
      int x = running[r];
      if (lat[x] > 0) { lat[x] -= dt; if (lat[x] < 1e-15) lat[x] = 0; still.push_back(x); continue; }
      remaining[x] -= rate[r] * dt;
      if (remaining[x] <= 1e-9 * std::max(1.0, work[x])) {
        done_at[x] = now;
        if (times) (*times)[2 * x + 1] = now;
        ++completed;
        active[ops[x].stream] = 0;
        ++head[ops[x].stream];
      } else {
        still.push_back(x);
      }
    }
    running.swap(still);
  }
  return now;
}

// ---- candidates ---------------------------------------------------------------------

static std::vector<int64_t> split_sizes(int64_t n, int64_t align, int max_parts) {
  std::set<int64_t> out;
  // block sizes are multiples of the kernel tile (or the whole extent when
  // it is smaller): a block narrower than a tile wastes most of the tile;
  // narrower powers of two are kept for budgets too small for a whole tile
  for (int parts = 1; parts <= max_parts; ++parts) {
    int64_t s = ceil_div(n, parts);
    if (align > 1) s = ceil_div(s, align) * align;
    out.insert(std::min(s, n));
  }
  for (int64_t s = 1; s < align && s < n; s *= 2) out.insert(s);
  return std::vector<int64_t>(out.begin(), out.end());
}

static std::vector<int64_t> panel_sizes(int64_t K) {
  std::set<int64_t> out;
  out.insert(K);
  if (K > kSplitMaxK) out.insert(kSplitMaxK);
  for (int64_t d = 2; d <= 64; d *= 2) {
    int64_t s = ceil_div(ceil_div(K, d), 64) * 64;
    if (s >= 256 && s < K) out.insert(s);
  }
  // short panels for budgets too small for longer ones
  for (int64_t s = 16; s < 256 && s < K; s *= 2) out.insert(s);
  return std::vector<int64_t>(out.begin(), out.end());
}

ooc_status plan_candidates(const Problem& pb, uint64_t budget_bytes, const ooc_opts* opts,
                           std::vector<ooc_plan_t>* plans, std::vector<double>* times) {
  plans->clear();
  times->clear();
  const int64_t M = pb.M, N = pb.N, K = pb.keff();
  const int prec = opts ? opts->precision : OOC_FP64;
  const int slices = (opts && opts->slices > 0) ? opts->slices : 6;
  const int want_streams = opts ? opts->nstreams : 0;
  const Machine& mc = machine();
  // lb: the analytic lower bound; tie: link plus kernel time, which orders
  // the many candidates of a link-bound problem that share one bound
  struct Cand { ooc_plan_t p; double lb, tie; };
  std::vector<Cand> cands;
  std::vector<int> stream_opts = {1, 2, 3};
  if (want_streams >= 1 && want_streams <= 3) stream_opts = {want_streams};
  double t_comp = 0.0;  // kernel-time bound of the current (mb, nb, kb)
  auto consider = [&](ooc_plan_t p) {
    Layout lay;
    p.precision = prec;
    p.slices = prec != OOC_FP64 ? slices : 0;
    // split tiles run K in panels of kSplitMaxK inside the kernel; plan panels
    // are kept to that size or below so both levels of panels coincide
    if (prec != OOC_FP64 && K > kSplitMaxK && p.kb > kSplitMaxK) return;
    if (plan_layout(pb, p, &lay) != OOC_OK) return;
    if (lay.bytes > budget_bytes) return;
    // analytic lower bound: operand traffic vs link, flops vs kernel rate
    const int64_t h = ceil_div(M, p.mb), w = ceil_div(N, p.nb);
    const int64_t P = K > 0 ? ceil_div(K, p.kb) : 1;
    double a_loads = 1, b_loads = 1;
    switch (p.order) {
      case OOC_ORDER_COLS: a_loads = (p.nbuf_a >= h * P) ? 1 : (double)w; b_loads = (P == 1 || p.nbuf_b >= P) ? 1 : (double)h; break;
      case OOC_ORDER_ROWS: b_loads = (p.nbuf_b >= w * P) ? 1 : (double)h; a_loads = (P == 1 || p.nbuf_a >= P) ? 1 : (double)w; break;
      case OOC_ORDER_COLS_P:
      case OOC_ORDER_COLS_PS: {
        const int64_t gs = p.group > 0 ? std::min<int64_t>(p.group, h) : h;
        a_loads = (double)w;
        // a backwards column reuses at most a group's panels of one K panel
        if (p.order == OOC_ORDER_COLS_PS) a_loads -= (double)(w - 1) * gs / ((double)P * h);
        b_loads = (P == 1 || p.nbuf_b >= P) ? 1 : (double)ceil_div(h, gs);
        break;
      }
      case OOC_ORDER_ROWS_P:
      case OOC_ORDER_ROWS_PS: {
        const int64_t gs = p.group > 0 ? std::min<int64_t>(p.group, w) : w;
        b_loads = (double)h;
        if (p.order == OOC_ORDER_ROWS_PS) b_loads -= (double)(h - 1) * gs / ((double)P * w);
        a_loads = (P == 1 || p.nbuf_a >= P) ? 1 : (double)ceil_div(w, gs);
        break;
      }
    }
    const bool c_moves = !pb.c_resident;
    const double h2d = 8.0 * ((double)M * K * a_loads + (double)K * N * b_loads +
                              (pb.beta != 0 && c_moves ? (double)M * N : 0));
    const double d2h = c_moves ? 8.0 * (double)M * N : 0.0;
    const double t_link = std::max(h2d / (mc.h2d_gbs * 1e9), d2h / (mc.d2h_gbs * 1e9));
    // the bound does not depend on the stream count: one entry per count
    for (int ns : stream_opts) {
      p.nstreams = ns;
      cands.push_back({p, std::max(t_link, t_comp), t_link + t_comp});
    }
  };
  const int max_parts = 64;
  std::vector<int64_t> mbs = split_sizes(M, 128, max_parts), nbs = split_sizes(N, 128, max_parts);
  std::vector<int64_t> kbs = K > 0 ? panel_sizes(K) : std::vector<int64_t>{0};
  for (int64_t mb : mbs) {
    for (int64_t nb : nbs) {
      const int64_t h = ceil_div(M, mb), w = ceil_div(N, nb);
      for (int64_t kb : kbs) {
        // kernel time from the tile model (full blocks plus the ragged edge
        // blocks), the same for every buffer and order variant below
        {
          const int64_t P = K > 0 ? ceil_div(K, kb) : 1;
          const int64_t mr = M - (h - 1) * mb, nr = N - (w - 1) * nb;
          const int64_t kr = K > 0 ? K - (P - 1) * kb : 0;
          auto kt = [&](int64_t m, int64_t n) {
            double t = (double)(P - 1) * kernel_seconds(mc, m, n, kb, prec, slices);
            return t + kernel_seconds(mc, m, n, kr, prec, slices);
          };
          t_comp = (double)(h - 1) * (w - 1) * kt(mb, nb) + (double)(h - 1) * kt(mb, nr) +
                   (double)(w - 1) * kt(mr, nb) + kt(mr, nr);
        }
        ooc_plan_t p{};
        p.mb = mb; p.nb = nb; p.kb = kb; p.nstreams = 3;
        const bool fullk = (K == 0 || kb >= K);
        // the paper's structure and its transpose (K whole)
        if (fullk) {
          for (int nbr : {1, 2}) {
            p.order = OOC_ORDER_COLS; p.nbuf_a = 2; p.nbuf_b = nbr; p.nbuf_c = 2; consider(p);
            p.order = OOC_ORDER_ROWS; p.nbuf_a = nbr; p.nbuf_b = 2; p.nbuf_c = 2; consider(p);
          }
          if (h > 1 && h <= 8) { p.order = OOC_ORDER_COLS; p.nbuf_a = (int)h; p.nbuf_b = 2; p.nbuf_c = 2; consider(p); }
          if (w > 1 && w <= 8) { p.order = OOC_ORDER_ROWS; p.nbuf_a = 2; p.nbuf_b = (int)w; p.nbuf_c = 2; consider(p); }
        } else {
          // C-stationary blocks with K panels streamed
          const int64_t P = ceil_div(K, kb);
          for (int nd : {0, 1}) {
            if (nd && (pb.beta == 0.0 || pb.lower)) continue;
            p.nbuf_d = nd;
            p.nbuf_a = 2; p.nbuf_b = 2; p.nbuf_c = 2;
            p.order = OOC_ORDER_COLS; consider(p);
            p.order = OOC_ORDER_ROWS; consider(p);
            // a block row's A panels (block column's B panels) resident, plus a
            // spare buffer so the next row's panels can arrive early
            if (P <= 16) {
              p.order = OOC_ORDER_ROWS; p.nbuf_a = (int)P + 1; p.nbuf_b = 2; consider(p);
              p.order = OOC_ORDER_COLS; p.nbuf_a = 2; p.nbuf_b = (int)P + 1; consider(p);
              p.nbuf_a = 2; p.nbuf_b = 2;
            }
            // a resident column (row) of C blocks, K panels outside; with the
            // initial C staged, no spare C buffer is needed at a column change
            if (h <= 64) { p.order = OOC_ORDER_COLS_P; p.nbuf_c = (int)h + (nd ? 0 : 1); consider(p); }
            if (w <= 64) { p.order = OOC_ORDER_ROWS_P; p.nbuf_c = (int)w + (nd ? 0 : 1); consider(p); }
            // small groups of C blocks walked K panel by K panel with the row's A
            // panels (column's B panels) resident: the last group of a row frees
            // its first panels a group's worth of tiles before the row ends, so
            // the next row's first panels arrive while the row finishes
            if (P <= 16) {
              for (int g : {2, 3, 4}) {
                for (int spare : {0, 1}) {
                  for (int stream_buf : {2, 3}) {  // buffers of the streamed operand
                    if (g < w) {
                      p.order = OOC_ORDER_ROWS_P; p.group = g; p.nbuf_a = (int)P + spare; p.nbuf_b = stream_buf;
                      p.nbuf_c = g + (nd ? 0 : 1); consider(p);
                    }
                    if (g < h) {
                      p.order = OOC_ORDER_COLS_P; p.group = g; p.nbuf_a = stream_buf; p.nbuf_b = (int)P + spare;
                      p.nbuf_c = g + (nd ? 0 : 1); consider(p);
                    }
                  }
                }
              }
              p.group = 0; p.nbuf_a = 2; p.nbuf_b = 2;
            }
          }
          p.nbuf_d = 0;
        }
      }
    }
  }
  if (cands.empty()) {
    // the paper's partition covers every budget its footprint rule allows
    ooc_plan_t pp{};
    if (paper_plan(pb, budget_bytes, &pp, prec, slices)) cands.push_back({pp, 0.0, 0.0});
  }
  if (cands.empty()) return fail(OOC_ERR_BUDGET, "no plan fits in the device budget");
  std::stable_sort(cands.begin(), cands.end(),
                   [](const Cand& a, const Cand& b) { return a.lb < b.lb || (a.lb == b.lb && a.tie < b.tie); });
  // simulate the most promising candidates, spread over host threads; fewer
  // for products that take milliseconds, where planning time would show, and
  // fewer when the schedules are long (about 3 million simulated operations
  // in total).  Results are collected in candidate order, so the choice is
  // deterministic.
  const bool small = 2.0 * (double)M * N * std::max<int64_t>(K, 1) < 1e11;
  size_t keep = std::min<size_t>(cands.size(), small ? 64 : 384);
  {
    double ops_total = 0.0;
    for (size_t c = 0; c < keep; ++c) {
      const ooc_plan_t& q = cands[c].p;
      const double tasks = (double)ceil_div(M, q.mb) * (double)ceil_div(N, q.nb) *
                           (double)(K > 0 ? ceil_div(K, q.kb) : 1);
      ops_total += 4.0 * tasks;
      if (ops_total > 3e6 && c >= 8) {
        keep = c;
        break;
      }
    }
  }
  std::vector<double> simt(keep, -1.0);
  auto work = [&](size_t first, size_t stride) {
    for (size_t c = first; c < keep; c += stride) {
      Layout lay;
      plan_layout(pb, cands[c].p, &lay);
      std::vector<ooc_op> ops;
      if (build_schedule(pb, cands[c].p, lay, &ops) != OOC_OK) continue;
      simt[c] = simulate(pb, cands[c].p, ops);
    }
  };
  const size_t nthreads = std::min<size_t>({(size_t)std::max(1u, std::thread::hardware_concurrency()), 8, keep});
  if (nthreads <= 1 || small) {
    work(0, 1);
  } else {
    std::vector<std::thread> pool;
    for (size_t t = 1; t < nthreads; ++t) pool.emplace_back(work, t, nthreads);
    work(0, nthreads);
    for (auto& th : pool) th.join();
  }
  std::vector<std::pair<double, ooc_plan_t>> sim;
  for (size_t c = 0; c < keep; ++c)
    if (simt[c] >= 0) sim.push_back({simt[c], cands[c].p});
  if (sim.empty()) return fail(OOC_ERR_BUDGET, "no schedulable plan fits in the device budget");
  std::stable_sort(sim.begin(), sim.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
  // the best _P plans walked backwards in every other row (column) as well:
  // the next row starts with the panels the last one ended with
  {
    std::vector<std::pair<double, ooc_plan_t>> more;
    size_t tried = 0;
    for (size_t c = 0; c < sim.size() && tried < 16; ++c) {
      ooc_plan_t q = sim[c].second;
      if (q.order != OOC_ORDER_COLS_P && q.order != OOC_ORDER_ROWS_P) continue;
      ++tried;
      q.order = q.order == OOC_ORDER_COLS_P ? OOC_ORDER_COLS_PS : OOC_ORDER_ROWS_PS;
      Layout lay;
      if (plan_layout(pb, q, &lay) != OOC_OK) continue;
      std::vector<ooc_op> ops;
      if (build_schedule(pb, q, lay, &ops) != OOC_OK) continue;
      more.push_back({simulate(pb, q, ops), q});
    }
    sim.insert(sim.end(), more.begin(), more.end());
    std::stable_sort(sim.begin(), sim.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
  }
  for (auto& s : sim) {
    plans->push_back(s.second);
    times->push_back(s.first);
  }
  return OOC_OK;
}

namespace {
// Plans already chosen, keyed by everything the choice depends on.
struct PlanKey {
  int64_t M, N, K;
  bool beta_nonzero;
  uint64_t budget;
  int planner, precision, slices, nstreams;
  bool c_resident;
  int64_t c_ld, base;
  bool transb, lower;
  bool operator<(const PlanKey& o) const {
    return std::tie(M, N, K, beta_nonzero, budget, planner, precision, slices, nstreams, c_resident, c_ld, base,
                    transb, lower) <
           std::tie(o.M, o.N, o.K, o.beta_nonzero, o.budget, o.planner, o.precision, o.slices, o.nstreams,
                    o.c_resident, o.c_ld, o.base, o.transb, o.lower);
  }
};
struct CachedPlan {
  ooc_plan_t plan;
  double predicted;
  bool declined;  // the learned planner's network declined the problem
};
std::mutex g_plan_mu;
std::map<PlanKey, CachedPlan> g_plan_cache;
}  // namespace

void clear_plan_cache() {
  std::lock_guard<std::mutex> lock(g_plan_mu);
  g_plan_cache.clear();
}

static ooc_status choose_plan_uncached(const Problem& pb, uint64_t budget_bytes, const ooc_opts* opts,
                                       ooc_plan_t* plan, double* predicted, bool* declined);

ooc_status choose_plan(const Problem& pb, uint64_t budget_bytes, const ooc_opts* opts, ooc_plan_t* plan,
                       double* predicted, bool* mlp_declined) {
  PlanKey key{pb.M, pb.N, pb.keff(), pb.beta != 0.0, budget_bytes,
              opts ? opts->planner : 0, opts ? opts->precision : 0, opts ? opts->slices : 0,
              opts ? opts->nstreams : 0, pb.c_resident, pb.c_ld, pb.base, pb.transb, pb.lower};
  {
    std::lock_guard<std::mutex> lock(g_plan_mu);
    auto it = g_plan_cache.find(key);
    if (it != g_plan_cache.end()) {
      *plan = it->second.plan;
      if (predicted) *predicted = it->second.predicted;
      if (mlp_declined) *mlp_declined = it->second.declined;
      return OOC_OK;
    }
  }
  double pred = 0.0;
  bool declined = false;
  ooc_status st = choose_plan_uncached(pb, budget_bytes, opts, plan, &pred, &declined);
  if (st != OOC_OK) return st;
  if (predicted) *predicted = pred;
  if (mlp_declined) *mlp_declined = declined;
  std::lock_guard<std::mutex> lock(g_plan_mu);
  if (g_plan_cache.size() > 4096) g_plan_cache.clear();
  g_plan_cache[key] = {*plan, pred, declined};
  return OOC_OK;
}

static ooc_status choose_plan_uncached(const Problem& pb, uint64_t budget_bytes, const ooc_opts* opts,
                                       ooc_plan_t* plan, double* predicted, bool* declined) {
  const int planner = opts ? opts->planner : OOC_PLAN_AUTO;
  if (planner == OOC_PLAN_PAPER) {
    const int prec = opts ? opts->precision : OOC_FP64;
    const int sl = (opts && opts->slices > 0) ? opts->slices : 6;
    if (!paper_plan(pb, budget_bytes, plan, prec, sl))
      return fail(OOC_ERR_BUDGET, "the paper's partitioner finds no split that fits the budget");
    Layout lay;
    ooc_status st = plan_layout(pb, *plan, &lay);
    if (st != OOC_OK) return st;
    if (lay.bytes > budget_bytes) return fail(OOC_ERR_BUDGET, "the paper's plan does not fit the budget with the split workspace");
    if (predicted) {
      std::vector<ooc_op> ops;
      build_schedule(pb, *plan, lay, &ops);
      *predicted = simulate(pb, *plan, ops);
    }
    return OOC_OK;
  }
  std::vector<ooc_plan_t> plans;
  std::vector<double> times;
  ooc_status st = plan_candidates(pb, budget_bytes, opts, &plans, &times);
  if (st != OOC_OK) return st;
  size_t best = 0;
  if (planner == OOC_PLAN_MLP) {
    // the network ranks the cost model's shortlist: the plans it was trained
    // on are among the model's best candidates plus a few random others, so
    // outside the shortlist its predictions would be extrapolations (and a
    // network trained on FP64 timings only declines split plans: the model's
    // choice stands)
    const size_t shortlist = std::min<size_t>(plans.size(), 8);
    std::vector<ooc_plan_t> top(plans.begin(), plans.begin() + shortlist);
    std::vector<double> pred;
    if (mlp_predict(pb, budget_bytes, top, &pred)) {
      for (size_t c = 1; c < pred.size(); ++c)
        if (pred[c] < pred[best]) best = c;
    } else {
      *declined = true;
    }
  }
  *plan = plans[best];
  if (predicted) *predicted = times[best];
  return OOC_OK;
}

}  // namespace ooc

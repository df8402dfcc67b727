// Checks of operation lists that a caller builds for the executor.
//
// The paper's programming model has the host drive the device through
// asynchronous copies, kernels, streams and events (Sections III-IV); the
// library's executor runs such a program given as an operation list
// (ooc_op).  Before it issues anything, every op of a caller's list is
// validated here against its host matrices and the device arena, so a
// malformed list is refused instead of reaching the device.  The ordering of
// ops is the caller's to get right; find_hazard reports the first pair of
// unordered ops that touch a common arena element, one of them writing it.
#include <algorithm>
#include <string>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"

namespace ooc {
namespace {

struct Region {
  int64_t off, rows, cols, ld;
};

bool empty(const Region& r) { return r.rows <= 0 || r.cols <= 0; }

// first and one-past-last element of a region
int64_t first_elem(const Region& r) { return r.off; }
int64_t end_elem(const Region& r) { return r.off + (r.rows - 1) * r.ld + r.cols; }

int64_t floor_div(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// whether two row-strided regions share an element (exact)
bool overlap(const Region& a, const Region& b) {
  if (empty(a) || empty(b)) return false;
  if (end_elem(a) <= first_elem(b) || end_elem(b) <= first_elem(a)) return false;
  const Region& p = a.rows <= b.rows ? a : b;  // walk the rows of the shorter one
  const Region& q = a.rows <= b.rows ? b : a;
  for (int64_t i = 0; i < p.rows; ++i) {
    const int64_t s = p.off + i * p.ld, e = s + p.cols;
    // rows j of q with q.off + j q.ld < e and q.off + j q.ld + q.cols > s
    int64_t jlo = floor_div(s - q.off - q.cols, q.ld) + 1, jhi = floor_div(e - q.off - 1, q.ld);
    jlo = std::max<int64_t>(jlo, 0);
    jhi = std::min<int64_t>(jhi, q.rows - 1);
    if (jlo <= jhi) return true;
  }
  return false;
}

// arena regions an op reads and writes
void regions(const ooc_op& o, std::vector<Region>* rd, std::vector<Region>* wr) {
  rd->clear();
  wr->clear();
  switch (o.kind) {
    case OOC_OP_H2D: wr->push_back({o.off_c, o.rows, o.cols, o.ld_c}); break;
    case OOC_OP_D2H: rd->push_back({o.off_c, o.rows, o.cols, o.ld_c}); break;
    case OOC_OP_GEMM:
    case OOC_OP_SPLIT_GEMM: {
      if (o.k > 0) {
        rd->push_back({o.off_a, o.rows, o.k, o.ld_a});
        if (o.flags & OOC_OPF_TRANSB) rd->push_back({o.off_b, o.cols, o.k, o.ld_b});
        else rd->push_back({o.off_b, o.k, o.cols, o.ld_b});
      }
      if (o.beta != 0.0) rd->push_back({o.off_c, o.rows, o.cols, o.ld_c});
      if (o.gamma != 0.0) rd->push_back({o.off_d, o.rows, o.cols, o.ld_d});
      wr->push_back({o.off_c, o.rows, o.cols, o.ld_c});
      if (o.kind == OOC_OP_SPLIT_GEMM && o.len_w > 0) {
        rd->push_back({o.off_w, 1, o.len_w, o.len_w});
        wr->push_back({o.off_w, 1, o.len_w, o.len_w});
      }
      break;
    }
    case OOC_OP_POTRF:
      rd->push_back({o.off_c, o.rows, o.rows, o.ld_c});
      rd->push_back({o.off_w, 1, 1, 1});
      wr->push_back({o.off_c, o.rows, o.rows, o.ld_c});
      wr->push_back({o.off_w, 1, 1, 1});
      break;
    case OOC_OP_TRSM:
      rd->push_back({o.off_a, o.cols, o.cols, o.ld_a});
      rd->push_back({o.off_c, o.rows, o.cols, o.ld_c});
      wr->push_back({o.off_c, o.rows, o.cols, o.ld_c});
      break;
    default: break;
  }
}

ooc_status bad_op(int64_t x, const std::string& what) {
  return fail(OOC_ERR_ARG, "op " + std::to_string(x) + ": " + what);
}

}  // namespace

ooc_status validate_ops(const ooc_op* ops, int64_t n, const ooc_host_matrix* mats, int nmats, int64_t arena_elems,
                        int precision, int slices, int* nstreams_out) {
  if (n < 0 || (n > 0 && !ops)) return fail(OOC_ERR_ARG, "no operation list");
  if (nmats < 0 || (nmats > 0 && !mats)) return fail(OOC_ERR_ARG, "no host matrices");
  for (int m = 0; m < nmats; ++m)
    if (mats[m].rows < 0 || mats[m].cols < 0 || mats[m].ld < mats[m].cols ||
        (mats[m].rows > 0 && mats[m].cols > 0 && !mats[m].ptr))
      return fail(OOC_ERR_ARG, "host matrix " + std::to_string(m) + " malformed");
  int ns = 1;
  std::vector<Region> rd, wr;
  int64_t prev_split = -1;  // the last SPLIT_GEMM op before x (slice reuse)
  for (int64_t x = 0; x < n; ++x) {
    const ooc_op& o = ops[x];
    if (o.kind < OOC_OP_H2D || o.kind > OOC_OP_TRSM) return bad_op(x, "unknown kind");
    if (o.stream < 0 || o.stream > 2) return bad_op(x, "stream must be 0, 1 or 2");
    ns = std::max(ns, o.stream + 1);
    if (o.nwait < 0 || o.nwait > OOC_MAX_WAITS) return bad_op(x, "nwait out of range");
    for (int k = 0; k < o.nwait; ++k)
      if (o.wait[k] < 0 || o.wait[k] >= x) return bad_op(x, "waits on an op that is not earlier in the list");
    if (o.rows < 0 || o.cols < 0 || o.k < 0) return bad_op(x, "negative extent");
    if (o.kind == OOC_OP_H2D || o.kind == OOC_OP_D2H) {
      if (o.mat < 0 || o.mat >= nmats) return bad_op(x, "host matrix index out of range");
      const ooc_host_matrix& hm = mats[o.mat];
      if (o.row0 < 0 || o.col0 < 0 || o.row0 + o.rows > hm.rows || o.col0 + o.cols > hm.cols)
        return bad_op(x, "copy outside its host matrix");
      if (o.ld_c < o.cols) return bad_op(x, "device leading dimension below the copy width");
    }
    if (o.kind == OOC_OP_GEMM || o.kind == OOC_OP_SPLIT_GEMM) {
      const int32_t known = o.kind == OOC_OP_GEMM ? (OOC_OPF_TRANSB | OOC_OPF_LOWER)
                                                  : (OOC_OPF_TRANSB | OOC_OPF_LOWER | OOC_OPF_REUSE_A | OOC_OPF_REUSE_B);
      if (o.flags & ~known) return bad_op(x, "unknown flags");
      if (o.ld_c < o.cols || (o.k > 0 && (o.ld_a < o.k || o.ld_b < ((o.flags & OOC_OPF_TRANSB) ? o.k : o.cols))) ||
          (o.gamma != 0.0 && o.ld_d < o.cols))
        return bad_op(x, "leading dimension below the block width");
      if (o.kind == OOC_OP_SPLIT_GEMM) {
        if (o.flags & OOC_OPF_LOWER) return bad_op(x, "lower-triangle products run in FP64 only");
        if (precision != OOC_SPLIT_BF16 && precision != OOC_SPLIT_INT8)
          return bad_op(x, "split product without a split precision in the options");
        if (slices < 1 || slices > 8) return bad_op(x, "split product needs 1..8 slices");
        if (o.k > 0 && (uint64_t)o.len_w * 8 < split_workspace_bytes(o.rows, o.cols, o.k, slices, slice_format(precision)))
          return bad_op(x, "split workspace too small");
        if (o.flags & (OOC_OPF_REUSE_A | OOC_OPF_REUSE_B)) {
          if (prev_split < 0) return bad_op(x, "slice reuse without an earlier split product");
          const ooc_op& p = ops[prev_split];
          if (p.rows != o.rows || p.cols != o.cols || p.k != o.k || o.k <= 0 || o.k > kSplitMaxK ||
              p.off_w != o.off_w || p.len_w != o.len_w || ((p.flags ^ o.flags) & OOC_OPF_TRANSB))
            return bad_op(x, "slice reuse needs the previous split product's extents, workspace and form");
          if ((o.flags & OOC_OPF_REUSE_A) && (p.off_a != o.off_a || p.ld_a != o.ld_a))
            return bad_op(x, "A slices reused from another panel");
          if ((o.flags & OOC_OPF_REUSE_B) && (p.off_b != o.off_b || p.ld_b != o.ld_b))
            return bad_op(x, "B slices reused from another panel");
        }
        prev_split = x;
      }
    }
    if (o.kind == OOC_OP_POTRF && o.ld_c < o.rows) return bad_op(x, "leading dimension below the block size");
    if (o.kind == OOC_OP_TRSM && (o.ld_c < o.cols || o.ld_a < o.cols))
      return bad_op(x, "leading dimension below the block width");
    if (o.kind == OOC_OP_TRSM && (o.flags & ~OOC_OPF_BACK)) return bad_op(x, "unknown flags");
    regions(o, &rd, &wr);
    for (const auto* v : {&rd, &wr})
      for (const Region& r : *v)
        if (!empty(r) && (r.off < 0 || end_elem(r) > arena_elems)) return bad_op(x, "operand outside the arena");
  }
  if (nstreams_out) *nstreams_out = ns;
  return OOC_OK;
}

bool find_hazard(const ooc_op* ops, int64_t n, int64_t* bx, int64_t* by) {
  // happens-before as bit sets: earlier ops of the same stream and waits, closed transitively
  const int64_t words = (n + 63) / 64;
  std::vector<uint64_t> reach((size_t)(n * words), 0);
  std::vector<int64_t> last(3, -1);
  for (int64_t x = 0; x < n; ++x) {
    uint64_t* rx = &reach[(size_t)(x * words)];
    auto add = [&](int64_t y) {
      const uint64_t* ry = &reach[(size_t)(y * words)];
      for (int64_t w = 0; w < words; ++w) rx[w] |= ry[w];
      rx[y / 64] |= 1ull << (y % 64);
    };
    const int s = ops[x].stream;
    if (s >= 0 && s < 3 && last[s] >= 0) add(last[s]);
    for (int k = 0; k < ops[x].nwait; ++k) add(ops[x].wait[k]);
    if (s >= 0 && s < 3) last[s] = x;
  }
  std::vector<std::vector<Region>> rds(n), wrs(n);
  for (int64_t x = 0; x < n; ++x) regions(ops[x], &rds[x], &wrs[x]);
  for (int64_t x = 0; x < n; ++x) {
    const uint64_t* rx = &reach[(size_t)(x * words)];
    for (int64_t y = 0; y < x; ++y) {
      if ((rx[y / 64] >> (y % 64)) & 1) continue;
      bool conflict = false;
      for (const Region& a : wrs[x]) {
        for (const Region& b : rds[y]) conflict = conflict || overlap(a, b);
        for (const Region& b : wrs[y]) conflict = conflict || overlap(a, b);
      }
      for (const Region& a : rds[x])
        for (const Region& b : wrs[y]) conflict = conflict || overlap(a, b);
      if (conflict) {
        *bx = x;
        *by = y;
        return true;
      }
    }
  }
  return false;
}

}  // namespace ooc

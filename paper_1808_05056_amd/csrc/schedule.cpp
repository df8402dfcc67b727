// Plan -> operation list.
//
// The pipeline of the paper (Section V, Figs. 2-4) moves A slices, B slices
// and C blocks into device buffers, multiplies, and moves C blocks back, with
// events that keep a buffer from being overwritten while an operation still
// reads it.  This builder generalises it: the C blocks (mb x nb) and K panels
// (kb) form a grid of tile tasks walked in a chosen order; each operand has a
// pool of device buffers; a panel stays resident until its buffer is needed
// again (a buffer whose content has no later use goes first, then the least
// recently used), and every reuse of a buffer waits for the last operation on
// each stream that read its old content.  A C block occupies a buffer from
// its first task until it is back on the host.  With the paper's configuration (order
// by columns, K not split, A and C double-buffered, B single-buffered, two
// streams by block parity) this reproduces the paper's ordering.
#include <algorithm>
#include <array>
#include <climits>
#include <map>
#include <set>
#include <string>

#include "internal.hpp"
#include "kernels.hpp"

namespace ooc {

int64_t ceil_div(int64_t a, int64_t b) { return b <= 0 ? 0 : (a + b - 1) / b; }

namespace {

struct Task {
  int64_t i, j, p;
};

struct Pool {
  int n = 0;
  std::vector<int64_t> key;       // content key per buffer (-1: empty)
  std::vector<int64_t> last_use;  // task index of the last use
  // op index of the last kernel on each stream that read the buffer's content
  // (a load into the buffer waits for all of them: with kernels on two
  // streams, the last reader's completion does not imply the other's)
  std::vector<std::array<int, 3>> readers;
  std::vector<int> load_op;       // op index that loaded the current content
  std::vector<int64_t> next_use;  // task index of the content's next use (INT64_MAX: none)
  void init(int nb) {
    n = nb;
    key.assign(nb, -1);
    last_use.assign(nb, -1);
    readers.assign(nb, {-1, -1, -1});
    load_op.assign(nb, -1);
    next_use.assign(nb, INT64_MAX);
  }
  int find(int64_t k) const {
    for (int s = 0; s < n; ++s)
      if (key[s] == k) return s;
    return -1;
  }
  // Buffer to overwrite for task t: an empty one; else, leaving out the buffer
  // the previous task read (its kernel is likely still running) unless it is
  // the only one, a buffer whose content is dead (least recently used first),
  // else the least recently used.
  int victim(int64_t t) const {
    for (int s = 0; s < n; ++s)
      if (key[s] < 0) return s;
    bool others = false;
    for (int s = 0; s < n; ++s)
      if (last_use[s] < t - 1) others = true;
    auto eligible = [&](int s) { return !others || last_use[s] < t - 1; };
    int best = -1;
    for (int s = 0; s < n; ++s)
      if (eligible(s) && next_use[s] == INT64_MAX && (best < 0 || last_use[s] < last_use[best])) best = s;
    if (best >= 0) return best;
    for (int s = 0; s < n; ++s)
      if (eligible(s) && (best < 0 || last_use[s] < last_use[best])) best = s;
    return best;
  }
};

// Tasks in walk order.  The _P orders walk groups of g C blocks of a block
// column (row) K panel by K panel, the blocks of a group inside; g = 0 means
// the whole column (row).  The _PS orders walk every other column (row)
// backwards (groups, K panels and blocks in reverse), so a column (row) starts
// with the group, the K panel and the block the previous one ended with, whose
// B (A) panels are still resident.
std::vector<Task> make_tasks(int order, int64_t h, int64_t w, int64_t P, int64_t g) {
  std::vector<Task> t;
  t.reserve((size_t)(h * w * P));
  switch (order) {
    case OOC_ORDER_COLS:
      for (int64_t j = 0; j < w; ++j)
        for (int64_t i = 0; i < h; ++i)
          for (int64_t p = 0; p < P; ++p) t.push_back({i, j, p});
      break;
    case OOC_ORDER_ROWS:
      for (int64_t i = 0; i < h; ++i)
        for (int64_t j = 0; j < w; ++j)
          for (int64_t p = 0; p < P; ++p) t.push_back({i, j, p});
      break;
    case OOC_ORDER_COLS_P:
    case OOC_ORDER_COLS_PS:
    case OOC_ORDER_ROWS_P:
    case OOC_ORDER_ROWS_PS: {
      // outer: block columns (COLS) or rows (ROWS); inner: the other index
      const bool cols = order == OOC_ORDER_COLS_P || order == OOC_ORDER_COLS_PS;
      const bool serp = order == OOC_ORDER_COLS_PS || order == OOC_ORDER_ROWS_PS;
      const int64_t no = cols ? w : h, ni = cols ? h : w;
      const int64_t gs = g > 0 ? std::min(g, ni) : ni;
      const int64_t ng = ceil_div(ni, gs);
      for (int64_t o = 0; o < no; ++o) {
        const bool rev = serp && (o & 1);
        for (int64_t gg = 0; gg < ng; ++gg) {
          const int64_t g0 = (rev ? ng - 1 - gg : gg) * gs, g1 = std::min(ni, g0 + gs);
          for (int64_t pp = 0; pp < P; ++pp) {
            const int64_t p = rev ? P - 1 - pp : pp;
            for (int64_t x = 0; x < g1 - g0; ++x) {
              const int64_t in = rev ? g1 - 1 - x : g0 + x;
              t.push_back(cols ? Task{in, o, p} : Task{o, in, p});
            }
          }
        }
      }
      break;
    }
  }
  return t;
}

// next_use[t] = index of the next task after t with the same key (INT64_MAX if none)
std::vector<int64_t> next_uses(const std::vector<int64_t>& keys) {
  std::vector<int64_t> nxt(keys.size(), INT64_MAX);
  std::map<int64_t, int64_t> seen;
  for (int64_t t = (int64_t)keys.size() - 1; t >= 0; --t) {
    auto it = seen.find(keys[t]);
    if (it != seen.end()) nxt[t] = it->second;
    seen[keys[t]] = t;
  }
  return nxt;
}

}  // namespace

void reorder_h2d(std::vector<ooc_op>* ops);

ooc_status build_schedule(const Problem& pb, const ooc_plan_t& plan, const Layout& lay,
                          std::vector<ooc_op>* ops_out) {
  std::vector<ooc_op>& ops = *ops_out;
  ops.clear();
  const int64_t M = pb.M, N = pb.N, K = pb.keff();
  if (M == 0 || N == 0) return OOC_OK;
  const int64_t mb = plan.mb, nb = plan.nb;
  const int64_t kb = K > 0 ? plan.kb : 0;
  const int64_t h = ceil_div(M, mb), w = ceil_div(N, nb);
  const int64_t P = K > 0 ? ceil_div(K, kb) : 1;
  const bool split = plan.precision != OOC_FP64 && K > 0;
  const int ns = plan.nstreams;

  std::vector<Task> tasks = make_tasks(plan.order, h, w, P, plan.group);
  // lower-triangle products: blocks wholly above the diagonal have no work
  // (the last row of block (i, j) lies above its first column)
  auto above = [&](int64_t i, int64_t j) { return std::min(M, (i + 1) * mb) - 1 < j * nb; };
  auto straddles = [&](int64_t i, int64_t j) { return !above(i, j) && i * mb < std::min(N, (j + 1) * nb) - 1; };
  if (pb.lower)
    tasks.erase(std::remove_if(tasks.begin(), tasks.end(), [&](const Task& tk) { return above(tk.i, tk.j); }),
                tasks.end());
  const int64_t T = (int64_t)tasks.size();
  if (T == 0) return OOC_OK;
  std::vector<int64_t> ka(T), kbk(T);
  for (int64_t t = 0; t < T; ++t) {
    ka[t] = tasks[t].i * P + tasks[t].p;
    kbk[t] = tasks[t].p * w + tasks[t].j;
  }
  std::vector<int64_t> nxa = next_uses(ka), nxb = next_uses(kbk);
  // a C block opens at its first task and goes home after its last (the _PS
  // orders walk K panels backwards in every other row or column)
  std::vector<char> opens(T, 0), closes(T, 0);
  {
    std::vector<int64_t> first(h * w, -1), last(h * w, -1);
    for (int64_t t = 0; t < T; ++t) {
      const int64_t ck = tasks[t].i * w + tasks[t].j;
      if (first[ck] < 0) first[ck] = t;
      last[ck] = t;
    }
    for (int64_t c = 0; c < h * w; ++c) {
      if (first[c] < 0) continue;  // skipped (above the diagonal)
      opens[first[c]] = 1;
      closes[last[c]] = 1;
    }
  }

  Pool pa, pbf, pd;
  pa.init(K > 0 ? plan.nbuf_a : 0);
  pbf.init(K > 0 ? plan.nbuf_b : 0);
  // staged initial C: the block starts from zero and beta*C_in is added at one
  // K-panel step, spread over the panels so the copies do not bunch up
  const bool staged = lay.nbufD > 0 && pb.beta != 0.0;
  pd.init(staged ? lay.nbufD : 0);
  // (position within its group * P) / group size for the _P orders
  auto spread = [&](int64_t x, int64_t n) {
    const int64_t gs = plan.group > 0 ? std::min<int64_t>(plan.group, n) : n;
    const int64_t x0 = (x / gs) * gs, len = std::min(n, x0 + gs) - x0;
    return ((x - x0) * P) / len;
  };
  auto fold_panel = [&](const Task& tk) -> int64_t {
    if (!staged || P == 1) return 0;
    if (plan.order == OOC_ORDER_COLS_P || plan.order == OOC_ORDER_COLS_PS) return spread(tk.i, h);
    if (plan.order == OOC_ORDER_ROWS_P || plan.order == OOC_ORDER_ROWS_PS) return spread(tk.j, w);
    return P - 1;
  };
  // resident C (accumulation sessions): blocks live at their place in the
  // resident matrix; only the op that last wrote each block is tracked
  const bool resident = pb.c_resident;
  std::vector<int> r_last_writer(resident ? h * w : 0, -1);
  // C bookkeeping: block key -> buffer, the op that last wrote it
  std::vector<int> c_close(plan.nbuf_c, -1);    // D2H op that emptied the buffer
  std::vector<int64_t> c_block(plan.nbuf_c, -1);  // open block key, -1 if free
  std::vector<int> c_last_writer(plan.nbuf_c, -1);
  std::vector<int64_t> c_closed_at(plan.nbuf_c, -1);

  auto stream_of = [&](int kind, int64_t task) -> int {
    if (ns == 3) return kind == OOC_OP_H2D ? 0 : (kind == OOC_OP_D2H ? 2 : 1);
    if (ns == 2) return (int)(task % 2);
    return 0;
  };
  // index of the last op on each stream (to drop waits already implied by stream order)
  auto push = [&](ooc_op op, std::vector<int> waits) -> int {
    op.stream = stream_of(op.kind, op.task);
    std::sort(waits.begin(), waits.end());
    waits.erase(std::unique(waits.begin(), waits.end()), waits.end());
    op.nwait = 0;
    for (int wv : waits) {
      if (wv < 0) continue;
      if (ops[wv].stream == op.stream) continue;  // earlier op on the same stream
      if (op.nwait >= OOC_MAX_WAITS) return -1;
      op.wait[op.nwait++] = wv;
    }
    ops.push_back(op);
    return (int)ops.size() - 1;
  };
  auto blank = [&](int kind, int64_t task) {
    ooc_op op{};
    op.kind = kind;
    op.task = (int32_t)task;
    return op;
  };

  int last_ws = -1;  // last split op, which used the (single) slice workspace
  int64_t prev_split = -1;  // its task
  for (int64_t t = 0; t < T; ++t) {
    const Task& tk = tasks[t];
    const int64_t i0 = tk.i * mb, m = std::min(mb, M - i0);
    const int64_t j0 = tk.j * nb, n = std::min(nb, N - j0);
    const int64_t k0 = tk.p * kb, k = K > 0 ? std::min(kb, K - k0) : 0;
    int sa = -1, sb = -1;
    // loads this task needs, issued in the order their buffers become free
    struct Load {
      ooc_op op;
      std::array<int, 3> war;  // kernels that read the buffer's old content
      int* load_op_slot;
      int last() const { return std::max(war[0], std::max(war[1], war[2])); }
    };
    std::vector<Load> loads;
    int c_load_placeholder = -1;
    if (K > 0) {
      // A panel (i, p)
      sa = pa.find(ka[t]);
      if (sa < 0) {
        sa = pa.victim(t);
        ooc_op op = blank(OOC_OP_H2D, t);
        op.mat = 0;
        op.slot = sa;
        op.row0 = i0; op.col0 = k0; op.rows = m; op.cols = k;
        op.off_c = lay.offA + sa * lay.slotA; op.ld_c = k;
        loads.push_back({op, pa.readers[sa], &pa.load_op[sa]});
        pa.readers[sa] = {-1, -1, -1};
        pa.key[sa] = ka[t];
      }
      pa.last_use[sa] = t;
      pa.next_use[sa] = nxa[t];
      // B panel (p, j)
      sb = pbf.find(kbk[t]);
      if (sb < 0) {
        sb = pbf.victim(t);
        ooc_op op = blank(OOC_OP_H2D, t);
        op.mat = 1;
        op.slot = sb;
        if (pb.transb) {  // rows j0.. of the stored B^T: the panel is kept n x k
          op.row0 = j0; op.col0 = k0; op.rows = n; op.cols = k;
          op.off_c = lay.offB + sb * lay.slotB; op.ld_c = k;
        } else {
          op.row0 = k0; op.col0 = j0; op.rows = k; op.cols = n;
          op.off_c = lay.offB + sb * lay.slotB; op.ld_c = n;
        }
        loads.push_back({op, pbf.readers[sb], &pbf.load_op[sb]});
        pbf.readers[sb] = {-1, -1, -1};
        pbf.key[sb] = kbk[t];
      }
      pbf.last_use[sb] = t;
      pbf.next_use[sb] = nxb[t];
    }
    // C block (i, j)
    const int64_t ckey = tk.i * w + tk.j;
    int sc = -1;
    if (!resident)
      for (int s = 0; s < plan.nbuf_c; ++s)
        if (c_block[s] == ckey) sc = s;
    int c_dep = -1;
    if (resident) {
      c_dep = r_last_writer[ckey];  // earlier K panels of the block, possibly on another stream
    } else if (opens[t]) {
      if (sc >= 0) return fail(OOC_ERR_ARG, "schedule: C block opened twice");
      for (int s = 0; s < plan.nbuf_c; ++s) {
        if (c_block[s] >= 0) continue;
        if (sc < 0 || c_closed_at[s] < c_closed_at[sc]) sc = s;
      }
      if (sc < 0)
        return fail(OOC_ERR_ARG, "plan has too few C buffers for its task order (nbuf_c=" +
                                     std::to_string(plan.nbuf_c) + ")");
      c_block[sc] = ckey;
      c_dep = c_close[sc];  // previous content must be home before it is overwritten
      // a lower-triangle product's block that straddles the diagonal is loaded
      // even with beta == 0: its elements above the diagonal go home unchanged
      if ((pb.beta != 0.0 && !staged) || (pb.lower && straddles(tk.i, tk.j))) {
        ooc_op op = blank(OOC_OP_H2D, t);
        op.mat = 2;
        op.slot = sc;
        op.row0 = i0; op.col0 = j0; op.rows = m; op.cols = n;
        op.off_c = lay.offC + sc * lay.slotC; op.ld_c = n;
        loads.push_back({op, {c_close[sc], -1, -1}, &c_load_placeholder});
      }
    } else {
      if (sc < 0) return fail(OOC_ERR_ARG, "schedule: C block not open");
      c_dep = c_last_writer[sc];
    }
    // staged initial C for this block, added at its fold panel
    int sd = -1;
    const bool fold_here = staged && tk.p == fold_panel(tk);
    if (fold_here) {
      sd = pd.victim(t);
      ooc_op op = blank(OOC_OP_H2D, t);
      op.mat = 2;
      op.slot = -1 - sd;
      op.row0 = i0; op.col0 = j0; op.rows = m; op.cols = n;
      op.off_c = lay.offD + sd * lay.slotD; op.ld_c = n;
      loads.push_back({op, pd.readers[sd], &pd.load_op[sd]});
      pd.readers[sd] = {-1, -1, -1};
      pd.key[sd] = ckey;
      pd.last_use[sd] = t;
    }
    std::stable_sort(loads.begin(), loads.end(), [](const Load& a, const Load& b) { return a.last() < b.last(); });
    for (Load& L : loads) {
      int x = push(L.op, {L.war[0], L.war[1], L.war[2]});
      if (x < 0) return fail(OOC_ERR_ARG, "schedule: too many waits");
      *L.load_op_slot = x;
    }
    if (c_load_placeholder >= 0) c_dep = c_load_placeholder;
    // the tile product
    ooc_op g = blank(split ? OOC_OP_SPLIT_GEMM : OOC_OP_GEMM, t);
    g.slot = sc;
    g.row0 = i0; g.col0 = j0; g.rows = m; g.cols = n;
    g.k0 = k0; g.k = k;
    if (K > 0) {
      g.off_a = lay.offA + sa * lay.slotA; g.ld_a = k;
      g.off_b = lay.offB + sb * lay.slotB; g.ld_b = pb.transb ? k : n;
    }
    g.flags = (pb.transb ? OOC_OPF_TRANSB : 0) | (pb.lower ? OOC_OPF_LOWER : 0);
    if (split && prev_split >= 0 && k <= kSplitMaxK) {
      // the previous split product left the slices of its panels in the
      // workspace: a panel it shares with this task (same extents) is not
      // sliced again
      const Task& pt = tasks[prev_split];
      const int64_t pm = std::min(mb, M - pt.i * mb), pn = std::min(nb, N - pt.j * nb);
      const int64_t pk = std::min(kb, K - pt.p * kb);
      if (pm == m && pn == n && pk == k) {
        if (ka[prev_split] == ka[t]) g.flags |= OOC_OPF_REUSE_A;
        if (kbk[prev_split] == kbk[t]) g.flags |= OOC_OPF_REUSE_B;
      }
    }
    if (resident) {
      g.slot = -1;
      g.off_c = i0 * pb.c_ld + j0;
      g.ld_c = pb.c_ld;
    } else {
      g.off_c = lay.offC + sc * lay.slotC;
      g.ld_c = n;
    }
    g.off_w = lay.offW; g.len_w = lay.lenW;
    g.alpha = pb.alpha;
    g.beta = opens[t] ? (staged ? 0.0 : pb.beta) : 1.0;
    g.gamma = 0.0;
    if (fold_here) {
      g.off_d = lay.offD + sd * lay.slotD;
      g.ld_d = n;
      g.gamma = pb.beta;
    }
    std::vector<int> gw = {c_dep};
    if (K > 0) {
      gw.push_back(pa.load_op[sa]);
      gw.push_back(pbf.load_op[sb]);
    }
    if (fold_here) gw.push_back(pd.load_op[sd]);
    if (split) gw.push_back(last_ws);
    int gx = push(g, gw);
    if (split) {
      last_ws = gx;
      prev_split = t;
    }
    if (gx < 0) return fail(OOC_ERR_ARG, "schedule: too many waits");
    if (K > 0) {
      pa.readers[sa][ops[gx].stream] = gx;
      pbf.readers[sb][ops[gx].stream] = gx;
    }
    if (fold_here) pd.readers[sd][ops[gx].stream] = gx;
    if (resident) {
      r_last_writer[ckey] = gx;
      continue;  // resident blocks stay on the device
    }
    c_last_writer[sc] = gx;
    // C block home after its last panel
    if (closes[t]) {
      ooc_op op = blank(OOC_OP_D2H, t);
      op.mat = 2;
      op.slot = sc;
      op.row0 = i0; op.col0 = j0; op.rows = m; op.cols = n;
      op.off_c = lay.offC + sc * lay.slotC; op.ld_c = n;
      int x = push(op, {gx});
      if (x < 0) return fail(OOC_ERR_ARG, "schedule: too many waits");
      c_close[sc] = x;
      c_block[sc] = -1;
      c_closed_at[sc] = t;
    }
  }
  if (ns == 3) reorder_h2d(&ops);
  return OOC_OK;
}

// With a stream of its own for host-to-device copies, the copies run in the
// order of the buffers they overwrite becoming free (the index of the kernel
// they wait for; copies into never-used buffers first), not in task order, so a
// copy whose buffer frees early is not held up behind one that must wait for a
// later kernel.  This cannot create a cycle: a copy's wait is on a kernel of an
// earlier task than the copy's own consumer.  The list is then re-emitted as a
// topological order of waits plus per-stream order, close to the original.
void reorder_h2d(std::vector<ooc_op>* ops_io) {
  std::vector<ooc_op>& ops = *ops_io;
  const int n = (int)ops.size();
  std::vector<int> h2d;
  for (int x = 0; x < n; ++x)
    if (ops[x].kind == OOC_OP_H2D) h2d.push_back(x);
  auto war = [&](int x) {
    int w = -1;
    for (int k = 0; k < ops[x].nwait; ++k) w = std::max(w, ops[x].wait[k]);
    return w;
  };
  std::stable_sort(h2d.begin(), h2d.end(), [&](int a, int b) { return war(a) < war(b); });
  // predecessors: waits, plus the previous op of the same stream in the new stream order
  std::vector<std::vector<int>> succ(n);
  std::vector<int> indeg(n, 0);
  auto edge = [&](int from, int to) {
    succ[from].push_back(to);
    ++indeg[to];
  };
  for (int x = 0; x < n; ++x)
    for (int k = 0; k < ops[x].nwait; ++k) edge(ops[x].wait[k], x);
  for (size_t q = 1; q < h2d.size(); ++q) edge(h2d[q - 1], h2d[q]);
  std::vector<int> last(4, -1);
  for (int x = 0; x < n; ++x) {
    if (ops[x].kind == OOC_OP_H2D) continue;
    int& l = last[ops[x].stream];
    if (l >= 0) edge(l, x);
    l = x;
  }
  // Kahn's algorithm, smallest original index first
  std::vector<int> order;
  order.reserve(n);
  std::set<int> ready;
  for (int x = 0; x < n; ++x)
    if (indeg[x] == 0) ready.insert(x);
  while (!ready.empty()) {
    const int x = *ready.begin();
    ready.erase(ready.begin());
    order.push_back(x);
    for (int y : succ[x])
      if (--indeg[y] == 0) ready.insert(y);
  }
  if ((int)order.size() != n) return;  // cannot happen (see above); keep the task order
  std::vector<int> pos(n);
  for (int q = 0; q < n; ++q) pos[order[q]] = q;
  std::vector<ooc_op> out(n);
  for (int q = 0; q < n; ++q) {
    ooc_op o = ops[order[q]];
    for (int k = 0; k < o.nwait; ++k) o.wait[k] = pos[o.wait[k]];
    out[q] = o;
  }
  ops.swap(out);
}

}  // namespace ooc

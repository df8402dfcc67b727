// Internal declarations of the out-of-core product library (host side).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "ooc.h"

namespace ooc {

// Thread-local error message behind ooc_last_error().
void set_error(const std::string& msg);
ooc_status fail(ooc_status st, const std::string& msg);

// Make `dev` the calling thread's current device, checking once that it is a
// gfx950 (OOC_ERR_NO_DEVICE otherwise).  Allocates nothing.
ooc_status use_device(int dev);

struct Problem {
  int64_t M = 0, N = 0, K = 0;
  double alpha = 1.0, beta = 0.0;
  // Accumulation sessions: with c_resident, C (M x N) already lives on the
  // device at element 0 of the arena with leading dimension c_ld; the plan
  // has no C buffers and moves no C, and its first K panel of each block
  // computes c = alpha*a*b + beta*c in place.  base: first arena element the
  // plan's own buffers may use (elements below it belong to resident C).
  bool c_resident = false;
  int64_t c_ld = 0;
  int64_t base = 0;
  // op(B) = B^T (B stored N x K); only the lower triangle of C (FP64 plans)
  bool transb = false;
  bool lower = false;
  // K as the pipeline sees it: 0 when alpha == 0 or K == 0 (A and B are not read).
  int64_t keff() const { return (alpha == 0.0 || K == 0) ? 0 : K; }
};

// Where the tile buffers live in the device arena (element offsets).
struct Layout {
  int64_t offA = 0, offB = 0, offC = 0, offD = 0, offW = 0;
  int64_t slotA = 0, slotB = 0, slotC = 0, slotD = 0;  // elements per buffer
  int nbufD = 0;                                        // staging buffers for initial C in use
  int64_t lenW = 0;                         // split workspace elements
  uint64_t bytes = 0;                       // whole arena
};

int64_t ceil_div(int64_t a, int64_t b);

// Checks a plan's shape and fills the arena layout. Returns OOC_OK or OOC_ERR_ARG.
ooc_status plan_layout(const Problem& pb, const ooc_plan_t& plan, Layout* lay);

// Split workspace elements a plan needs (0 for FP64 plans).
int64_t split_workspace_elems(const Problem& pb, const ooc_plan_t& plan);

// The operation list of a plan (see ooc_op). Returns OOC_OK or OOC_ERR_ARG
// (e.g. too few C buffers for the task order).
ooc_status build_schedule(const Problem& pb, const ooc_plan_t& plan, const Layout& lay,
                          std::vector<ooc_op>* ops);

// The paper's partitioner (Section V); false if nothing fits.
bool paper_partition(int64_t M, int64_t N, int64_t K, uint64_t budget_elems, int64_t* h, int64_t* w);

// The plan the paper's MMOOC runs for a problem (two streams, A and C
// double-buffered, B single-buffered), with the given tile precision.
bool paper_plan(const Problem& pb, uint64_t budget_bytes, ooc_plan_t* plan, int precision, int slices);

// Hardware figures the cost model uses.
// Measured on an MI355X (PCIe Gen5 x16 host link, pinned host memory).
struct Machine {
  double h2d_gbs = 56.6;          // pinned host -> device, one direction active (GB/s, 2-D copies)
  double d2h_gbs = 57.1;          // device -> pinned host
  double duplex_h2d_gbs = 56.5;   // host -> device while device -> host is active
  double duplex_d2h_gbs = 47.3;   // device -> host while host -> device is active
  double copy_latency_s = 12e-6;
  double kernel_tflops = 72.85;    // FP64 tile kernel, two workgroups per CU, large k
  double kernel_tflops_1wg = 38.0; // same with one workgroup per CU
  double kernel_k0 = 30.0;         // per-tile fixed cost in units of k
  double kernel_scalar_factor = 1.15;  // odd leading dimensions (8-byte loads)
  double kernel_launch_s = 6e-6;
  double split_tflops_per_product = 1080.0;  // BF16 slice-product rate (TFLOP/s of BF16 work), 256 x 128 tiles,
                                             // one per CU, slice-sum traffic excluded (8192^3 launches at s = 5)
  double split_k0 = 160.0;                  // per weight and tile: pipeline start in units of k
  double int8_tops_per_product = 2090.0;    // INT8 slice-product rate (TOP/s), same tiles (1.99x the BF16 rate)
  double int8_wide_tops_per_product = 2200.0;  // same on 256 x 256 tiles (1.05x)
  double hbm_bytes_per_s = 5e12;            // streaming rate of the split kernel's slice-sum tile
  int cus = 256;
};
const Machine& machine();

// Simulated time of an operation list under the cost model.
// If times is not null it receives the start and end of every op.
double simulate(const Problem& pb, const ooc_plan_t& plan, const std::vector<ooc_op>& ops,
                std::vector<double>* times = nullptr);

// Candidate plans (feasible within the budget) with modelled times, best first.
ooc_status plan_candidates(const Problem& pb, uint64_t budget_bytes, const ooc_opts* opts,
                           std::vector<ooc_plan_t>* plans, std::vector<double>* times);

// Choose a plan according to opts->planner (the measured sweep is not done
// here: OOC_PLAN_SWEEP gets the cost model's choice).  With the learned
// planner, *mlp_declined (if given) tells whether its network declined the
// problem, so that the cost model's choice stands.
ooc_status choose_plan(const Problem& pb, uint64_t budget_bytes, const ooc_opts* opts,
                       ooc_plan_t* plan, double* predicted, bool* mlp_declined = nullptr);

// Forget cached plan choices (after a new planner network is loaded).
void clear_plan_cache();

// Operation lists given by a caller (oplist.cpp): validation against the
// host matrices and the arena (OOC_ERR_ARG naming the first bad op; the
// stream count the list uses in *nstreams_out), and the first pair of
// unordered ops (x > y) that touch a common arena element, one writing it.
ooc_status validate_ops(const ooc_op* ops, int64_t n, const ooc_host_matrix* mats, int nmats, int64_t arena_elems,
                        int precision, int slices, int* nstreams_out);
bool find_hazard(const ooc_op* ops, int64_t n, int64_t* x, int64_t* y);

// MLP planner hook: predicted times for candidate plans, or false if no model is loaded.
bool mlp_predict(const Problem& pb, uint64_t budget_bytes, const std::vector<ooc_plan_t>& plans,
                 std::vector<double>* seconds);

}  // namespace ooc

// The FP64 tile kernel configuration the library launches (see
// dgemm_f64_kernel.hpp for the kernel).
#include "dgemm_f64_kernel.hpp"
#include "kernels.hpp"

namespace ooc {

hipError_t launch_dgemm_f64(int64_t m, int64_t n, int64_t k, double alpha, const double* A, int64_t lda,
                            const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                            double gamma, const double* D, int64_t ldd, hipStream_t stream, bool transb,
                            int64_t tri) {
  // 128 x 128 tiles, 4 waves of 64 x 64, K steps of 16, two workgroups per CU;
  // a wave raises its priority while it issues its block of matrix
  // instructions, so that of the two waves sharing a SIMD the one with MFMAs
  // ready keeps the matrix unit busy while the other loads and stores (66 ->
  // 72.7 TFLOP/s on 8192 x 4096 x 16384)
  if (transb)
    return dgemm::launch<128, 128, 16, 2, 2, 2, dgemm::GROUP_M, true, false, true>(m, n, k, alpha, A, lda, B, ldb,
                                                                                   beta, C, ldc, gamma, D, ldd, tri,
                                                                                   stream);
  return dgemm::launch<128, 128, 16, 2, 2, 2, dgemm::GROUP_M, true, false>(m, n, k, alpha, A, lda, B, ldb, beta, C,
                                                                            ldc, gamma, D, ldd, tri, stream);
}

}  // namespace ooc

// Setup kernel: the exponential-kernel covariance in integration order
// (Section 3.2: Sigma_pq = variance exp(-|x_p - x_q| / range), plus an
// optional nugget on the diagonal), written column-major.
#include "internal.hpp"

namespace tlrqmc {

__global__ __launch_bounds__(256) void k_cov_exp(int64_t n, const double *xy, double inv_range,
                                                 double variance, double nugget, double *A, int64_t lda,
                                                 int64_t col0) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const int64_t j = col0 + blockIdx.y;
  if (i >= n) return;
  const double dx = xy[2 * i] - xy[2 * j];
  const double dy = xy[2 * i + 1] - xy[2 * j + 1];
  double v = variance * exp(-sqrt(dx * dx + dy * dy) * inv_range);
  if (i == j) v += nugget;
  A[j * lda + i] = v;
}

void launch_cov_exp(hipStream_t s, int64_t n, const double *xy_perm, double range, double variance,
                    double nugget, double *A, int64_t lda, int64_t col0, int64_t ncols) {
  for (int64_t c = 0; c < ncols; c += 65535) {
    const int64_t nc = ncols - c < 65535 ? ncols - c : 65535;
    hipLaunchKernelGGL(k_cov_exp, dim3(static_cast<unsigned>((n + 255) / 256), static_cast<unsigned>(nc)),
                       dim3(256), 0, s, n, xy_perm, 1.0 / range, variance, nugget, A, lda, col0 + c);
  }
}

}  // namespace tlrqmc

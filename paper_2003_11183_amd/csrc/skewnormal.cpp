// Skew-normal likelihood client (Section 5: the stochastic generator
// Z = xi 1 + A X + B |Y| of Eq. 5 and its density, Eq. 6):
//
//   log f(z) = n log 2 + log phi_n(z - xi 1; A A^T + B B^T)
//              + log Phi_n(-inf, c; Gamma),
//   C = A^-1 B,  Gamma = (I + C^T C)^-1,  c = Gamma C^T A^-1 (z - xi 1),
//
// with A the lower Cholesky factor of sigma1^2 exp(-|h|/beta1) and B the
// covariance matrix sigma2^2 exp(-|h|/beta2) (Section 5.2).  The dense
// linear algebra runs on the device (rocSOLVER / rocBLAS); Gamma stays on
// the device and is factored into the TLR form, and the MVN probability term
// is the library's estimator.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <memory>
#include <vector>

#include "internal.hpp"

namespace tlrqmc {
void launch_cov_exp(hipStream_t s, int64_t n, const double *xy_perm, double range, double variance,
                    double nugget, double *A, int64_t lda, int64_t col0, int64_t ncols);
void launch_set_identity(hipStream_t s, double *A, int64_t lda, int64_t n);
}  // namespace tlrqmc

using namespace tlrqmc;

extern "C" {

int tlrqmc_skewnormal_loglik(tlrqmc_ctx *ctx, int64_t n, const double *xy, const double *z,
                             const tlrqmc_skewnormal_params *prm, int m, double tol, int max_rank, int order,
                             const tlrqmc_qmc_opts *opts, tlrqmc_skewnormal_result *out, double *c_out,
                             tlrqmc_factor **factor_out) {
  clear_error();
  if (!ctx || !xy || !z || !prm || !opts || !out) return fail(TLRQMC_EINVAL, "null argument");
  if (factor_out) *factor_out = nullptr;
  if (n < 1 || m < 1) return fail(TLRQMC_EINVAL, "n and m must be >= 1");
  if (!(prm->sigma1 > 0.0) || !(prm->beta1 > 0.0) || !(prm->sigma2 >= 0.0) || !(prm->beta2 > 0.0) ||
      !std::isfinite(prm->xi))
    return fail(TLRQMC_EINVAL, "need sigma1 > 0, beta1 > 0, sigma2 >= 0, beta2 > 0 and a finite xi");
  if (order != 0 && order != 2) return fail(TLRQMC_EINVAL, "order must be 0 (geometric) or 2 (during Cholesky)");
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(z[i]) || !std::isfinite(xy[2 * i]) || !std::isfinite(xy[2 * i + 1]))
      return fail(TLRQMC_EINVAL, "non-finite observation or location at %lld", static_cast<long long>(i));
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(TLRQMC_EDEVICE, "hipSetDevice failed");
  std::memset(out, 0, sizeof *out);
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  hipStream_t s = ctx->stream;
  const int64_t lda = round_up(n, 64);
  std::vector<double> r(n), t(n), c(n), dg(n), a(n, -INFINITY);
  tlrqmc_factor *F = nullptr;
  int st;
  auto t1 = t0, t2 = t0;
  {
  // dense buffers of the linear algebra, released before the estimator runs
  Scratch sc(ctx);
  double *K1 = sc.get<double>(static_cast<size_t>(lda) * n);
  double *B = sc.get<double>(static_cast<size_t>(lda) * n);
  double *W = sc.get<double>(static_cast<size_t>(lda) * n);
  double *dxy = sc.get<double>(2 * n);
  double *dr = sc.get<double>(n), *dt = sc.get<double>(n), *ds = sc.get<double>(n);
  if (!K1 || !B || !W || !dxy || !dr || !dt || !ds) return fail(TLRQMC_ENOMEM, "device allocation failed");
  rocblas_handle h = blas_handle(ctx);
  if (!h) return fail(TLRQMC_EDEVICE, "rocblas_create_handle failed");
  for (int64_t i = 0; i < n; ++i) r[i] = z[i] - prm->xi;
  if (hipMemcpyAsync(dxy, xy, 2 * n * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(dr, r.data(), n * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess)
    return fail(TLRQMC_EDEVICE, "copy of the inputs failed");
  {
    SharedDevice dev;
    launch_cov_exp(s, n, dxy, prm->beta1, prm->sigma1 * prm->sigma1, 0.0, K1, lda, 0, n);
    launch_cov_exp(s, n, dxy, prm->beta2, prm->sigma2 * prm->sigma2, 0.0, B, lda, 0, n);
    if (hipStreamSynchronize(s) != hipSuccess) return fail(TLRQMC_EDEVICE, "covariance kernels failed");
  }
  const rocblas_int N = static_cast<rocblas_int>(n), LD = static_cast<rocblas_int>(lda);
  const double one = 1.0, zero = 0.0;
  // Omega = K1 + B B^T and its Cholesky factor: log det and the quadratic form
  if (hipMemcpy2DAsync(W, lda * sizeof(double), K1, lda * sizeof(double), n * sizeof(double), n,
                       hipMemcpyDeviceToDevice, s) != hipSuccess)
    return fail(TLRQMC_EDEVICE, "copy failed");
  {
    ExclusiveDevice dev;
    if (!dev.ok ||
        rocblas_dsyrk(h, rocblas_fill_lower, rocblas_operation_none, N, N, &one, B, LD, &one, W, LD) !=
            rocblas_status_success ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(TLRQMC_EDEVICE, "rocBLAS syrk failed");
  }
  if ((st = device_cholesky(ctx, W, lda, n))) return st;
  if (hipMemcpyAsync(dt, dr, n * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess) return fail(TLRQMC_EDEVICE, "copy failed");
  {
    ExclusiveDevice dev;
    if (!dev.ok ||
        rocblas_dtrsv(h, rocblas_fill_lower, rocblas_operation_none, rocblas_diagonal_non_unit, N, W, LD, dt, 1) !=
            rocblas_status_success ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(TLRQMC_EDEVICE, "rocBLAS trsv failed");
  }
  // read back through pinned memory: a strided copy into pageable memory was
  // not always complete when the stream synchronization returned
  double *hp = ctx->pinned(4, 2 * n * sizeof(double));
  if (!hp) return fail(TLRQMC_ENOMEM, "pinned host allocation failed");
  if (hipMemcpy2DAsync(hp, sizeof(double), W, (lda + 1) * sizeof(double), sizeof(double), n, hipMemcpyDeviceToHost,
                       s) != hipSuccess ||
      hipMemcpyAsync(hp + n, dt, n * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(TLRQMC_EDEVICE, "copy failed");
  std::memcpy(dg.data(), hp, n * sizeof(double));
  std::memcpy(t.data(), hp + n, n * sizeof(double));
  double logdet = 0.0, quad = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    logdet += 2.0 * std::log(dg[i]);
    quad += t[i] * t[i];
  }
  out->log_density = -0.5 * (static_cast<double>(n) * std::log(2.0 * M_PI) + logdet + quad);
  // A = chol(K1); C = A^-1 B; G = I + C^T C; c = G^-1 C^T A^-1 r; Gamma = G^-1
  if ((st = device_cholesky(ctx, K1, lda, n))) return st;
  if (hipMemcpyAsync(dt, dr, n * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess) return fail(TLRQMC_EDEVICE, "copy failed");
  {
    SharedDevice dev;
    launch_set_identity(s, W, lda, n);
    if (hipStreamSynchronize(s) != hipSuccess) return fail(TLRQMC_EDEVICE, "identity kernel failed");
  }
  {
    ExclusiveDevice dev;
    if (!dev.ok) return fail(TLRQMC_EDEVICE, "device synchronize failed");
    if (rocblas_dtrsm(h, rocblas_side_left, rocblas_fill_lower, rocblas_operation_none, rocblas_diagonal_non_unit, N,
                      N, &one, K1, LD, B, LD) != rocblas_status_success ||
        rocblas_dsyrk(h, rocblas_fill_lower, rocblas_operation_transpose, N, N, &one, B, LD, &one, W, LD) !=
            rocblas_status_success ||
        rocblas_dtrsv(h, rocblas_fill_lower, rocblas_operation_none, rocblas_diagonal_non_unit, N, K1, LD, dt, 1) !=
            rocblas_status_success ||
        rocblas_dgemv(h, rocblas_operation_transpose, N, N, &one, B, LD, dt, 1, &zero, ds, 1) !=
            rocblas_status_success ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(TLRQMC_EDEVICE, "rocBLAS update failed");
  }
  if ((st = device_cholesky(ctx, W, lda, n))) return st;
  {
    rocblas_int *dinfo = sc.get<rocblas_int>(1);
    rocblas_int info = 0;
    ExclusiveDevice dev;
    if (!dinfo || !dev.ok ||
        rocblas_dtrsv(h, rocblas_fill_lower, rocblas_operation_none, rocblas_diagonal_non_unit, N, W, LD, ds, 1) !=
            rocblas_status_success ||
        rocblas_dtrsv(h, rocblas_fill_lower, rocblas_operation_transpose, rocblas_diagonal_non_unit, N, W, LD, ds,
                      1) != rocblas_status_success ||
        rocsolver_dpotri(h, rocblas_fill_lower, N, W, LD, dinfo) != rocblas_status_success ||
        hipMemcpyAsync(hp + n, dinfo, sizeof info, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(hp, ds, n * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess || (std::memcpy(&info, hp + n, sizeof info), info != 0))
      return fail(TLRQMC_EDEVICE, "inverse of I + C^T C failed");
    std::memcpy(c.data(), hp, n * sizeof(double));
  }
  if (c_out) std::memcpy(c_out, c.data(), n * sizeof(double));
  t1 = clk::now();
  // the MVN probability term: Gamma (on the device) in TLR form, then the estimator
  if ((st = factor_from_device_dense(ctx, n, W, lda, a.data(), c.data(), xy, m, tol, max_rank, order, nullptr, &F)) < 0)
    return st;
  t2 = clk::now();
  }
  std::unique_ptr<tlrqmc_factor, void (*)(tlrqmc_factor *)> fguard(F, tlrqmc_factor_free);
  if ((st = mvn_prob(ctx, F, a.data(), c.data(), opts, &out->prob)) < 0) return st;
  const auto t3 = clk::now();
  out->log_prob = out->prob.log_p;
  out->log_prob_std_err = out->prob.std_err;
  out->log_prob_rel_err = out->prob.rel_err;
  out->loglik = static_cast<double>(n) * std::log(2.0) + out->log_density + out->log_prob;
  out->seconds[0] = std::chrono::duration<double>(t1 - t0).count();
  out->seconds[1] = std::chrono::duration<double>(t2 - t1).count();
  out->seconds[2] = std::chrono::duration<double>(t3 - t2).count();
  if (factor_out) *factor_out = fguard.release();
  return TLRQMC_OK;
}

}  // extern "C"

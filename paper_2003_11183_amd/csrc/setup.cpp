// Setup of the estimator (not on the timed path): geometric order, block
// reordering and the TLR Cholesky factor.
//
// * Geometric order (Section 3.2): Morton order of the locations.
// * Block reordering (Section 3.3, "Block reordering" algorithm): each block
//   scored by univariate conditioning (Trinh and Genz 2015), blocks sorted
//   ascending by selection with swaps, variables inside a block in the
//   order the conditioning chose.
// * TLR factor (Sections 3.3-3.4): dense Cholesky of the permuted
//   covariance on the device (blocked right-looking: host POTRF of the
//   diagonal block, rocBLAS TRSM and SYRK for the panel and the trailing
//   matrix), then each off-diagonal tile truncated on the host to the
//   singular values above tol: column-pivoted Householder QR (Businger and
//   Golub 1965) down to a residual far below tol, then a one-sided Jacobi
//   SVD (Hestenes 1958) of the small triangular factor.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <numeric>
#include <vector>

#include "internal.hpp"
#include "setup_kernels.hpp"

namespace tlrqmc {

namespace {

// ------------------------------------------------------------------ Morton
uint64_t spread16(uint64_t v) {
  v &= 0xFFFF;
  uint64_t out = 0;
  for (int bit = 0; bit < 16; ++bit) out |= ((v >> bit) & 1ull) << (2 * bit);
  return out;
}

void morton(int64_t n, const double *xy, int32_t *perm) {
  std::vector<uint64_t> key(n, 0);
  for (int ax = 0; ax < 2; ++ax) {
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t i = 0; i < n; ++i) {
      lo = std::min(lo, xy[2 * i + ax]);
      hi = std::max(hi, xy[2 * i + ax]);
    }
    for (int64_t i = 0; i < n; ++i) {
      uint64_t qi = 0;
      if (hi > lo) qi = static_cast<uint64_t>(std::floor((xy[2 * i + ax] - lo) / (hi - lo) * 65535.0 + 0.5));
      key[i] |= ax == 0 ? (spread16(qi) << 1) : spread16(qi);
    }
  }
  std::vector<int32_t> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int32_t x, int32_t y) { return key[x] < key[y]; });
  std::copy(idx.begin(), idx.end(), perm);
}

// Covariance entry (p, q) in original indexing.
double cov_entry(const tlrqmc_cov *c, int64_t p, int64_t q) {
  if (c->kind == 0) return c->sigma[q * c->ld + p];
  const double dx = c->xy[2 * p] - c->xy[2 * q];
  const double dy = c->xy[2 * p + 1] - c->xy[2 * q + 1];
  double v = c->variance * std::exp(-std::sqrt(dx * dx + dy * dy) / c->range);
  if (p == q) v += c->nugget;
  return v;
}

int check_cov(int64_t n, const tlrqmc_cov *c) {
  if (!c) return fail(TLRQMC_EINVAL, "null covariance");
  if (c->kind == 0) {
    if (!c->sigma || c->ld < n) return fail(TLRQMC_EINVAL, "dense covariance needs sigma and ld >= n");
  } else if (c->kind == 1) {
    if (!c->xy) return fail(TLRQMC_EINVAL, "kernel covariance needs locations");
    if (!(c->range > 0.0) || !(c->variance > 0.0) || !(c->nugget >= 0.0))
      return fail(TLRQMC_EINVAL, "range and variance must be > 0, nugget >= 0");
    for (int64_t i = 0; i < 2 * n; ++i)
      if (!std::isfinite(c->xy[i])) return fail(TLRQMC_EINVAL, "non-finite location");
  } else {
    return fail(TLRQMC_EINVAL, "unknown covariance kind %d", c->kind);
  }
  return TLRQMC_OK;
}

double Phi(double x) { return 0.5 * std::erfc(-x * M_SQRT1_2); }
double phi(double x) { return std::isfinite(x) ? std::exp(-0.5 * x * x) * 0.39894228040143267794 : 0.0; }

// Univariate conditioning of one block: chosen order and log of the score;
// y_out (optional) receives the truncated means of the whitened variables in
// that order.
double univariate_conditioning(int m, std::vector<double> &S, std::vector<double> &a, std::vector<double> &b,
                               std::vector<int> &order, std::vector<double> *y_out = nullptr) {
  std::vector<double> L(static_cast<size_t>(m) * m, 0.0), y(m, 0.0);
  order.resize(m);
  std::iota(order.begin(), order.end(), 0);
  auto Sat = [&](int i, int j) -> double & { return S[static_cast<size_t>(i) * m + j]; };
  auto Lat = [&](int i, int j) -> double & { return L[static_cast<size_t>(i) * m + j]; };
  double logp = 0.0;
  std::vector<double> at(m), bt(m), sd(m), pr(m);
  for (int i = 0; i < m; ++i) {
    int best = i;
    for (int j = i; j < m; ++j) {
      double s = 0.0, v = Sat(j, j);
      for (int k = 0; k < i; ++k) {
        s += Lat(j, k) * y[k];
        v -= Lat(j, k) * Lat(j, k);
      }
      sd[j] = std::sqrt(std::max(v, 0.0));
      at[j] = (a[j] - s) / sd[j];
      bt[j] = (b[j] - s) / sd[j];
      pr[j] = Phi(bt[j]) - Phi(at[j]);
      if (pr[j] < pr[best]) best = j;
    }
    if (best != i) {
      for (int k = 0; k < m; ++k) std::swap(Sat(i, k), Sat(best, k));
      for (int k = 0; k < m; ++k) std::swap(Sat(k, i), Sat(k, best));
      for (int k = 0; k < m; ++k) std::swap(Lat(i, k), Lat(best, k));
      std::swap(a[i], a[best]);
      std::swap(b[i], b[best]);
      std::swap(order[i], order[best]);
      std::swap(at[i], at[best]);
      std::swap(bt[i], bt[best]);
      std::swap(sd[i], sd[best]);
      std::swap(pr[i], pr[best]);
    }
    const double lii = sd[i];
    Lat(i, i) = lii;
    for (int j = i + 1; j < m; ++j) {
      double s = Sat(j, i);
      for (int k = 0; k < i; ++k) s -= Lat(j, k) * Lat(i, k);
      Lat(j, i) = s / lii;
    }
    if (pr[i] > 0.0) {
      y[i] = (phi(at[i]) - phi(bt[i])) / pr[i];
      logp += std::log(pr[i]);
    } else {
      y[i] = std::isfinite(bt[i]) ? bt[i] : (std::isfinite(at[i]) ? at[i] : 0.0);
      logp = -INFINITY;
    }
  }
  if (y_out) *y_out = y;
  return logp;
}

// ------------------------------------------------------- tile compression
// Truncated SVD of the mi x mj column-major tile T (leading dimension ldt):
// keeps the singular values > tol (at most cap when cap > 0).  Writes U
// (mi x k, row-major, columns scaled by the singular values) and V
// (mj x k, row-major); returns k and sets capped.  Column-pivoted
// Householder QR T P = Q R stops once the trailing columns' norm drops
// below tol / 1000; the singular values and right vectors of R then come
// from the eigen-decomposition of the small Gram matrix R R^T (cyclic
// Jacobi), so the work past the QR grows with the rank, not the tile.
int compress_tile(const double *T, int64_t ldt, int mi, int mj, double tol, int cap, std::vector<double> &U,
                  std::vector<double> &V, bool &capped) {
  capped = false;
  std::vector<double> A(static_cast<size_t>(mi) * mj);
  for (int c = 0; c < mj; ++c)
    for (int rr = 0; rr < mi; ++rr) A[static_cast<size_t>(c) * mi + rr] = T[c * ldt + rr];
  auto Aat = [&](int rr, int c) -> double & { return A[static_cast<size_t>(c) * mi + rr]; };
  std::vector<int> piv(mj);
  std::iota(piv.begin(), piv.end(), 0);
  std::vector<double> cn(mj);
  const int kmax = std::min(mi, mj);
  std::vector<double> tau;
  const double stop = 1e-3 * tol;
  int kq = 0;
  // squared norms of the trailing columns, updated after each reflection
  // and recomputed where the update has cancelled most of the value
  std::vector<double> cn0(mj);
  for (int c = 0; c < mj; ++c) {
    double s = 0.0;
    for (int rr = 0; rr < mi; ++rr) s += Aat(rr, c) * Aat(rr, c);
    cn[c] = cn0[c] = s;
  }
  for (; kq < kmax; ++kq) {
    double rest = 0.0;
    int best = kq;
    for (int c = kq; c < mj; ++c) {
      if (kq > 0) {
        const double r = Aat(kq - 1, c);
        cn[c] -= r * r;
        if (!(cn[c] > 1e-8 * cn0[c])) {
          double s = 0.0;
          for (int rr = kq; rr < mi; ++rr) s += Aat(rr, c) * Aat(rr, c);
          cn[c] = cn0[c] = s;
        }
      }
      rest += cn[c];
      if (cn[c] > cn[best]) best = c;
    }
    if (std::sqrt(rest) <= stop) break;
    if (best != kq) {
      for (int rr = 0; rr < mi; ++rr) std::swap(Aat(rr, kq), Aat(rr, best));
      std::swap(piv[kq], piv[best]);
      std::swap(cn[kq], cn[best]);
      std::swap(cn0[kq], cn0[best]);
    }
    // Householder reflector for column kq, rows kq..mi-1
    double nrm = 0.0;
    for (int rr = kq; rr < mi; ++rr) nrm += Aat(rr, kq) * Aat(rr, kq);
    nrm = std::sqrt(nrm);
    const double alpha = Aat(kq, kq) >= 0 ? -nrm : nrm;
    const double v0 = Aat(kq, kq) - alpha;
    double vnorm2 = v0 * v0;
    for (int rr = kq + 1; rr < mi; ++rr) vnorm2 += Aat(rr, kq) * Aat(rr, kq);
    double t = 0.0;
    if (vnorm2 > 0.0) {
      t = 2.0 / vnorm2;
      Aat(kq, kq) = v0;  // keep v in the column for now
      for (int c = kq + 1; c < mj; ++c) {
        double d = 0.0;
        for (int rr = kq; rr < mi; ++rr) d += Aat(rr, kq) * Aat(rr, c);
        d *= t;
        for (int rr = kq; rr < mi; ++rr) Aat(rr, c) -= d * Aat(rr, kq);
      }
    }
    tau.push_back(t);
    // store v below the diagonal (scaled so v0 = 1), R diagonal = alpha
    if (vnorm2 > 0.0) {
      for (int rr = kq + 1; rr < mi; ++rr) Aat(rr, kq) /= v0;
      tau.back() = t * v0 * v0;
    }
    Aat(kq, kq) = alpha;
  }
  const int kq_final = kq;
  int k = 0;
  if (kq_final > 0) {
    // G = R^T (mj x kq) with its rows in the original column order, and the
    // kq x kq Gram matrix M = G^T G = R R^T, diagonalized by cyclic Jacobi
    // rotations: M = J diag(lambda) J^T, sigma = sqrt(lambda).
    std::vector<double> G(static_cast<size_t>(mj) * kq_final, 0.0), J(static_cast<size_t>(kq_final) * kq_final, 0.0),
        M(static_cast<size_t>(kq_final) * kq_final, 0.0);
    auto Gat = [&](int rr, int c) -> double & { return G[static_cast<size_t>(c) * mj + rr]; };
    auto Jat = [&](int rr, int c) -> double & { return J[static_cast<size_t>(c) * kq_final + rr]; };
    auto Mat = [&](int rr, int c) -> double & { return M[static_cast<size_t>(c) * kq_final + rr]; };
    for (int c = 0; c < kq_final; ++c) {
      Jat(c, c) = 1.0;
      for (int col = c; col < mj; ++col) Gat(piv[col], c) = Aat(c, col);
    }
    for (int p = 0; p < kq_final; ++p)
      for (int q = p; q < kq_final; ++q) {
        double d = 0.0;
        for (int col = std::max(p, q); col < mj; ++col) d += Aat(p, col) * Aat(q, col);
        Mat(p, q) = d;
        Mat(q, p) = d;
      }
    // A pair is rotated unless |M_pq| is negligible against sqrt(M_pp M_qq):
    // R is graded by the pivoting, and this relative test keeps the small
    // singular values accurate too.
    for (int sweep = 0; sweep < 60; ++sweep) {
      double off = 0.0;
      for (int p = 0; p < kq_final - 1; ++p)
        for (int q = p + 1; q < kq_final; ++q) {
          const double apq = Mat(p, q);
          const double rel = std::sqrt(Mat(p, p) * Mat(q, q));
          if (!(std::fabs(apq) > 1e-17 * rel)) continue;
          off = std::max(off, std::fabs(apq) / rel);
          const double theta = (Mat(q, q) - Mat(p, p)) / (2.0 * apq);
          const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(1.0 + theta * theta));
          const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = t * cs;
          for (int rr = 0; rr < kq_final; ++rr) {  // columns p, q
            const double mp = Mat(rr, p), mq = Mat(rr, q);
            Mat(rr, p) = cs * mp - sn * mq;
            Mat(rr, q) = sn * mp + cs * mq;
          }
          for (int cc = 0; cc < kq_final; ++cc) {  // rows p, q
            const double mp = Mat(p, cc), mq = Mat(q, cc);
            Mat(p, cc) = cs * mp - sn * mq;
            Mat(q, cc) = sn * mp + cs * mq;
          }
          for (int rr = 0; rr < kq_final; ++rr) {
            const double jp = Jat(rr, p), jq = Jat(rr, q);
            Jat(rr, p) = cs * jp - sn * jq;
            Jat(rr, q) = sn * jp + cs * jq;
          }
        }
      if (off < 1e-17) break;
    }
    // sigma_c = sqrt(lambda_c); the right vectors G J_c / sigma_c are formed
    // below for the kept columns only
    std::vector<std::pair<double, int>> sv(kq_final);
    for (int c = 0; c < kq_final; ++c) sv[c] = {std::sqrt(std::max(Mat(c, c), 0.0)), c};
    std::sort(sv.begin(), sv.end(), [](const auto &x, const auto &y) {
      return x.first > y.first || (x.first == y.first && x.second < y.second);
    });
    while (k < kq_final && sv[k].first > tol) ++k;
    if (cap > 0 && k > cap) {
      k = cap;
      capped = true;
    }
    // Q (mi x kq) from the reflectors, applied to the chosen columns of J:
    // U = Q J(:, idx) (times sigma), V = G J(:, idx) / sigma.
    U.assign(static_cast<size_t>(mi) * k, 0.0);
    V.assign(static_cast<size_t>(mj) * k, 0.0);
    std::vector<double> w(mi);
    for (int c = 0; c < k; ++c) {
      const int src = sv[c].second;
      const double s = sv[c].first;
      std::fill(w.begin(), w.end(), 0.0);
      for (int rr = 0; rr < kq_final; ++rr) w[rr] = Jat(rr, src) * s;
      for (int h = kq_final - 1; h >= 0; --h) {
        if (tau[h] == 0.0) continue;
        double d = w[h];
        for (int rr = h + 1; rr < mi; ++rr) d += Aat(rr, h) * w[rr];
        d *= tau[h];
        w[h] -= d;
        for (int rr = h + 1; rr < mi; ++rr) w[rr] -= d * Aat(rr, h);
      }
      for (int rr = 0; rr < mi; ++rr) U[static_cast<size_t>(rr) * k + c] = w[rr];
      for (int rr = 0; rr < mj; ++rr) {
        double g = 0.0;
        for (int r2 = 0; r2 < kq_final; ++r2) g += Gat(rr, r2) * Jat(r2, src);
        V[static_cast<size_t>(rr) * k + c] = g / s;
      }
    }
  } else {
    U.clear();
    V.clear();
  }
  return k;
}

}  // namespace

void release_blas(tlrqmc_ctx *ctx) {
  if (ctx->blas) (void)rocblas_destroy_handle(static_cast<rocblas_handle>(ctx->blas));
  ctx->blas = nullptr;
}

// Kernel building the permuted covariance (kernels_setup.hip).
void launch_cov_exp(hipStream_t s, int64_t n, const double *xy_perm, double range, double variance,
                    double nugget, double *A, int64_t lda, int64_t col0, int64_t ncols);
void launch_gather_sym(hipStream_t s, const double *S, int64_t lds, const int32_t *p, double *A, int64_t lda,
                       int64_t n);
// Kernels of the block reordering during the Cholesky factorization.
void launch_pack_diag(hipStream_t s, const double *A, int64_t lda, int64_t j0, int m, int mb, int count,
                      double *out);
void launch_permute_rows(hipStream_t s, double *A, int64_t lda, int64_t n, int64_t j0, int nrows,
                         const int32_t *rows, const int32_t *src, const int32_t *slot, double *tmp);

}  // namespace tlrqmc

namespace tlrqmc {
namespace {

using clk = std::chrono::steady_clock;
double secs(clk::time_point a, clk::time_point b) { return std::chrono::duration<double>(b - a).count(); }

thread_local int t_shared_depth = 0;  // shared holds of the device lock by this thread

// The context's rocBLAS handle on its stream (created on first use).
rocblas_handle blas_of(tlrqmc_ctx *ctx) {
  if (!ctx->blas) {
    rocblas_handle nh;
    if (rocblas_create_handle(&nh) != rocblas_status_success) return nullptr;
    // no atomics: the factor (and so every estimate) is reproducible bit for bit
    rocblas_set_atomics_mode(nh, rocblas_atomics_not_allowed);
    ctx->blas = nh;
  }
  rocblas_handle h = static_cast<rocblas_handle>(ctx->blas);
  rocblas_set_stream(h, ctx->stream);
  return h;
}

// Validated permutation, or the geometric order (Morton for locations,
// identity for a dense matrix) when perm is null.
int order_of(int64_t n, const tlrqmc_cov *cov, const int32_t *perm, std::vector<int32_t> &p) {
  p.resize(n);
  if (perm) {
    std::vector<uint8_t> seen(n, 0);
    for (int64_t i = 0; i < n; ++i) {
      if (perm[i] < 0 || perm[i] >= n || seen[perm[i]]) return fail(TLRQMC_EINVAL, "perm is not a permutation");
      seen[perm[i]] = 1;
      p[i] = perm[i];
    }
  } else if (cov->kind == 1) {
    morton(n, cov->xy, p.data());
  } else {
    std::iota(p.begin(), p.end(), 0);
  }
  return TLRQMC_OK;
}

// The covariance in order p on the device, column-major, leading dimension lda.
int build_cov(tlrqmc_ctx *ctx, int64_t n, const tlrqmc_cov *cov, const std::vector<int32_t> &p, double *A,
              int64_t lda) {
  hipStream_t s = ctx->stream;
  // covariance in integration order, column-major
  if (cov->kind == 1) {
    std::vector<double> xyp(2 * n);
    for (int64_t i = 0; i < n; ++i) {
      xyp[2 * i] = cov->xy[2 * p[i]];
      xyp[2 * i + 1] = cov->xy[2 * p[i] + 1];
    }
    double *dxy = static_cast<double *>(ctx->dmalloc(2 * n * sizeof(double)));
    if (!dxy) return fail(TLRQMC_ENOMEM, "device allocation failed");
    hipError_t e;
    {
      SharedDevice dev;
      hipMemcpyAsync(dxy, xyp.data(), 2 * n * sizeof(double), hipMemcpyHostToDevice, s);
      launch_cov_exp(s, n, dxy, cov->range, cov->variance, cov->nugget, A, lda, 0, n);
      e = hipStreamSynchronize(s);
    }
    ctx->dfree(dxy);
    if (e != hipSuccess) return fail(TLRQMC_EDEVICE, "covariance kernel failed");
  } else {
    std::vector<double> col(n);
    for (int64_t j = 0; j < n; ++j) {
      for (int64_t i = 0; i < n; ++i) col[i] = cov->sigma[static_cast<int64_t>(p[j]) * cov->ld + p[i]];
      if (hipMemcpy(A + j * lda, col.data(), n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        return fail(TLRQMC_EDEVICE, "copy of the covariance failed");
    }
  }
  return TLRQMC_OK;
}

// Dense Cholesky (lower) of the n x n matrix A on the device, by this
// library's kernels (kernels_chol.hip): they run beside the estimator
// kernels like any other (shared device lock).
int device_potrf(tlrqmc_ctx *ctx, int64_t n, double *A, int64_t lda, int64_t col0, int m) {
  int32_t *dinfo = static_cast<int32_t *>(ctx->dmalloc(sizeof(int32_t)));
  double *scratch = static_cast<double *>(ctx->dmalloc(kCholScratch * sizeof(double)));
  auto release = [&] {
    ctx->dfree(dinfo);
    ctx->dfree(scratch);
  };
  if (!dinfo || !scratch) {
    release();
    return fail(TLRQMC_ENOMEM, "device allocation failed");
  }
  int32_t *hinfo = reinterpret_cast<int32_t *>(ctx->pinned(5, sizeof(int32_t)));
  if (!hinfo) {
    release();
    return fail(TLRQMC_ENOMEM, "pinned host allocation failed");
  }
  hipStream_t s = ctx->stream;
  bool ok;
  {
    SharedDevice dev;
    ok = hipMemsetAsync(dinfo, 0, sizeof(int32_t), s) == hipSuccess;
    if (ok) {
      launch_cholesky(s, A, lda, n, dinfo, scratch);
      ok = hipGetLastError() == hipSuccess &&
           hipMemcpyAsync(hinfo, dinfo, sizeof(int32_t), hipMemcpyDeviceToHost, s) == hipSuccess &&
           hipStreamSynchronize(s) == hipSuccess;
    }
  }
  const int32_t info = ok ? *hinfo : 0;
  release();
  if (!ok) return fail(TLRQMC_EDEVICE, "Cholesky failed on the device");
  if (info > 0)
    return fail(TLRQMC_ENOTSPD, "covariance not positive definite at column %lld (tile %lld)",
                static_cast<long long>(col0 + info - 1), static_cast<long long>((col0 + info - 1) / m));
  return TLRQMC_OK;
}

// From the dense factor L (lower part of A, order p) to the TLR factor:
// download by panels, compress the off-diagonal tiles, build the layouts.
// Device compression (kernels_compress.hip) in batches of tiles: the factor
// stays on the device; only the diagonal tiles and the packed U and V blocks
// come back.  A tile whose QR needs more than kCmpKq steps is downloaded and
// compressed on the host.
int compress_build_device(tlrqmc_ctx *ctx, double *A, int64_t lda, int64_t n, int m, const std::vector<int32_t> &p,
                          double tol, int max_rank, double *phase,
                          std::unique_ptr<double, std::function<void(double *)>> &Aguard, tlrqmc_factor **out) {
  hipStream_t s = ctx->stream;
  const int r = static_cast<int>((n + m - 1) / m);
  std::vector<int> tm(r);
  for (int i = 0; i < r; ++i) tm[i] = static_cast<int>(std::min<int64_t>(m, n - static_cast<int64_t>(i) * m));
  std::vector<int64_t> doff(r + 1, 0);
  for (int i = 0; i < r; ++i) doff[i + 1] = doff[i] + static_cast<int64_t>(tm[i]) * tm[i];
  const int64_t ntiles = static_cast<int64_t>(r) * (r - 1) / 2;
  const int64_t B = std::max<int64_t>(1, compress_batch_tiles(n, m));
  const int64_t wslot = static_cast<int64_t>(m) * m, vslot = compress_vslot(m);
  Scratch sc(ctx);
  double *dW = sc.get<double>(B * wslot);
  double *dV = sc.get<double>(B * vslot);
  double *dOut = sc.get<double>(B * 2 * vslot);
  int32_t *dInfo = sc.get<int32_t>(B * 4);
  int32_t *hInfo = reinterpret_cast<int32_t *>(ctx->pinned(7, B * 4 * sizeof(int32_t)));
  double *hDiag = ctx->pinned(8, doff[r] * sizeof(double));
  if (!dW || !dV || !dOut || !dInfo) return fail(TLRQMC_ENOMEM, "device allocation for the compression failed");
  if (!hInfo || !hDiag) return fail(TLRQMC_ENOMEM, "pinned host staging allocation failed");
  const auto t_dl = clk::now();
  {
    SharedDevice dev;
    bool ok = true;
    for (int i = 0; i < r && ok; ++i) {
      const int64_t c0 = static_cast<int64_t>(i) * m;
      ok = hipMemcpy2DAsync(hDiag + doff[i], tm[i] * sizeof(double), A + c0 * lda + c0, lda * sizeof(double),
                            tm[i] * sizeof(double), tm[i], hipMemcpyDeviceToHost, s) == hipSuccess;
    }
    if (!ok || hipStreamSynchronize(s) != hipSuccess) return fail(TLRQMC_EDEVICE, "copy of the diagonal tiles failed");
  }
  std::vector<double> hdiag(doff[r]);
#pragma omp parallel for schedule(dynamic, 1)
  for (int i = 0; i < r; ++i)
    for (int t = 0; t < tm[i]; ++t)
      for (int u = 0; u < tm[i]; ++u)
        hdiag[doff[i] + static_cast<int64_t>(t) * tm[i] + u] =
            u <= t ? hDiag[doff[i] + static_cast<int64_t>(u) * tm[i] + t] : 0.0;
  const auto t_cp = clk::now();
  phase[1] += secs(t_dl, t_cp);
  std::vector<int32_t> ranks(static_cast<size_t>(r) * r, 0);
  // U and V of each tile: in the copy of its batch's packed output (batch,
  // offset of U, offset of V), or in a vector of its own when compressed on
  // the host
  std::vector<std::vector<double>> batch_uv;
  struct Src {
    int32_t batch = -1;
    int64_t uo = 0, vo = 0;
  };
  std::vector<Src> src(static_cast<size_t>(ntiles));
  std::vector<int64_t> left;  // tiles for the host
  std::vector<std::vector<double>> Ul, Vl;
  int cap_hits = 0;
  for (int64_t t0 = 0; t0 < ntiles; t0 += B) {
    const int count = static_cast<int>(std::min<int64_t>(B, ntiles - t0));
    {
      SharedDevice dev;
      launch_compress(s, A, lda, n, m, t0, count, tol, max_rank, dW, dV, dOut, dInfo);
      if (hipGetLastError() != hipSuccess ||
          hipMemcpyAsync(hInfo, dInfo, count * 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return fail(TLRQMC_EDEVICE, "tile compression failed on the device");
    }
    int64_t ut = 0, vt = 0;
    for (int q = 0; q < count; ++q) {
      int64_t r0, c0;
      int mi, mj;
      compress_tile_at(t0 + q, n, m, r0, c0, mi, mj);
      const int k = (hInfo[4 * q + 2] & 1) ? 0 : hInfo[4 * q + 1];
      ut += static_cast<int64_t>(mi) * k;
      vt += static_cast<int64_t>(mj) * k;
    }
    double *hOut = ctx->pinned(6, std::max<int64_t>(1, ut + vt) * sizeof(double));
    if (!hOut) return fail(TLRQMC_ENOMEM, "pinned host staging allocation failed");
    if (ut + vt > 0) {
      SharedDevice dev;
      if (hipMemcpyAsync(hOut, dOut, (ut + vt) * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return fail(TLRQMC_EDEVICE, "copy of the compressed tiles failed");
    }
    const int32_t bi = static_cast<int32_t>(batch_uv.size());
    batch_uv.emplace_back(hOut, hOut + ut + vt);
    int64_t uo = 0, vo = ut;
    for (int q = 0; q < count; ++q) {
      const int64_t t = t0 + q;
      int64_t r0, c0;
      int mi, mj;
      compress_tile_at(t, n, m, r0, c0, mi, mj);
      const int i = static_cast<int>(r0 / m), j = static_cast<int>(c0 / m);
      if (hInfo[4 * q + 2] & 1) {
        left.push_back(t);
        continue;
      }
      const int k = hInfo[4 * q + 1];
      ranks[static_cast<size_t>(i) * r + j] = k;
      cap_hits += (hInfo[4 * q + 2] & 2) ? 1 : 0;
      src[t] = {bi, uo, vo};
      uo += static_cast<int64_t>(mi) * k;
      vo += static_cast<int64_t>(mj) * k;
    }
  }
  if (!left.empty()) {
    // tiles beyond the device kernels' QR depth: download and compress here
    const size_t per = static_cast<size_t>(m) * m;
    double *hT = ctx->pinned(9, left.size() * per * sizeof(double));
    if (!hT) return fail(TLRQMC_ENOMEM, "pinned host staging allocation failed");
    {
      SharedDevice dev;
      bool ok = true;
      for (size_t q = 0; q < left.size() && ok; ++q) {
        int64_t r0, c0;
        int mi, mj;
        compress_tile_at(left[q], n, m, r0, c0, mi, mj);
        ok = hipMemcpy2DAsync(hT + q * per, mi * sizeof(double), A + c0 * lda + r0, lda * sizeof(double),
                              mi * sizeof(double), mj, hipMemcpyDeviceToHost, s) == hipSuccess;
      }
      if (!ok || hipStreamSynchronize(s) != hipSuccess) return fail(TLRQMC_EDEVICE, "copy of the factor failed");
    }
    int hits = 0;
    Ul.resize(left.size());
    Vl.resize(left.size());
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : hits)
    for (size_t q = 0; q < left.size(); ++q) {
      int64_t r0, c0;
      int mi, mj;
      compress_tile_at(left[q], n, m, r0, c0, mi, mj);
      bool capped = false;
      const int k = compress_tile(hT + q * per, mi, mi, mj, tol, max_rank, Ul[q], Vl[q], capped);
      ranks[static_cast<size_t>(r0 / m) * r + c0 / m] = k;
      hits += capped ? 1 : 0;
    }
    cap_hits += hits;
    for (size_t q = 0; q < left.size(); ++q) src[left[q]].batch = -2 - static_cast<int32_t>(q);
  }
  phase[2] += secs(t_cp, clk::now());
  Aguard.reset();
  const auto t_layout = clk::now();
  // the exchange arrays, tiles in row order, filled in parallel
  std::vector<int64_t> uoff(ntiles + 1, 0), voff(ntiles + 1, 0);
  for (int64_t t = 0; t < ntiles; ++t) {
    int64_t r0, c0;
    int mi, mj;
    compress_tile_at(t, n, m, r0, c0, mi, mj);
    const int64_t k = ranks[static_cast<size_t>(r0 / m) * r + c0 / m];
    uoff[t + 1] = uoff[t] + mi * k;
    voff[t + 1] = voff[t] + mj * k;
  }
  std::vector<double> hU(uoff[ntiles]), hV(voff[ntiles]);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t t = 0; t < ntiles; ++t) {
    const Src &e = src[t];
    const int64_t nu = uoff[t + 1] - uoff[t], nv = voff[t + 1] - voff[t];
    const double *su, *sv;
    if (e.batch >= 0) {
      su = batch_uv[e.batch].data() + e.uo;
      sv = batch_uv[e.batch].data() + e.vo;
    } else {
      su = Ul[-2 - e.batch].data();
      sv = Vl[-2 - e.batch].data();
    }
    if (nu) std::memcpy(hU.data() + uoff[t], su, nu * sizeof(double));
    if (nv) std::memcpy(hV.data() + voff[t], sv, nv * sizeof(double));
  }
  std::vector<std::vector<double>>().swap(batch_uv);
  int st = factor_build_take(ctx, n, m, p.data(), hdiag, ranks.data(), hU, hV, cap_hits, out);
  if (st) return st;
  phase[3] = secs(t_layout, clk::now());
  for (int k = 0; k < 4; ++k) (*out)->setup_seconds[k] = phase[k];
  (*out)->host_tiles = static_cast<int64_t>(left.size());
  return cap_hits > 0 ? TLRQMC_WARN_RANKCAP : TLRQMC_OK;
}

int compress_build(tlrqmc_ctx *ctx, double *A, int64_t lda, int64_t n, int m, const std::vector<int32_t> &p,
                   double tol, int max_rank, double *phase, std::unique_ptr<double, std::function<void(double *)>> &Aguard,
                   tlrqmc_factor **out) {
  hipStream_t s = ctx->stream;
  int st;
  if (m <= kCmpMaxTile && n > m)
    return compress_build_device(ctx, A, lda, n, m, p, tol, max_rank, phase, Aguard, out);
  // Column panels of L go to the host in groups, through two pinned staging
  // buffers: the copy of the next group overlaps the compression of this
  // one.  Every off-diagonal tile of a group is compressed in one parallel
  // loop (tiles are independent).
  const int r = static_cast<int>((n + m - 1) / m);
  std::vector<int> tm(r);
  for (int i = 0; i < r; ++i) tm[i] = static_cast<int>(std::min<int64_t>(m, n - static_cast<int64_t>(i) * m));
  std::vector<int64_t> doff(r + 1, 0), poff(r + 1, 0);
  for (int i = 0; i < r; ++i) doff[i + 1] = doff[i] + static_cast<int64_t>(tm[i]) * tm[i];
  for (int j = 0; j < r; ++j) poff[j + 1] = poff[j] + (n - static_cast<int64_t>(j) * m) * tm[j];
  const int64_t stage_doubles = std::max<int64_t>(poff[1], int64_t{32} << 20);  // >= 256 MB or the first panel
  double *stage[2] = {ctx->pinned(0, stage_doubles * 8), ctx->pinned(1, stage_doubles * 8)};
  if (!stage[0] || !stage[1]) return fail(TLRQMC_ENOMEM, "pinned host staging allocation failed");
  std::vector<std::pair<int, int>> groups;  // [j0, j1)
  for (int j0 = 0; j0 < r;) {
    int j1 = j0 + 1;
    while (j1 < r && poff[j1 + 1] - poff[j0] <= stage_doubles) ++j1;
    groups.push_back({j0, j1});
    j0 = j1;
  }
  std::vector<double> hdiag(doff[r]);
  std::vector<int32_t> ranks(static_cast<size_t>(r) * r, 0);
  std::vector<std::vector<double>> Us(static_cast<size_t>(r) * r), Vs(static_cast<size_t>(r) * r);
  int cap_hits = 0;
  Events evs;
  auto download = [&](size_t g) {
    const int j0 = groups[g].first, j1 = groups[g].second;
    double *dst = stage[g % 2];
    for (int j = j0; j < j1; ++j) {
      const int64_t c0 = static_cast<int64_t>(j) * m, rows = n - c0;
      if (hipMemcpy2DAsync(dst + (poff[j] - poff[j0]), rows * sizeof(double), A + c0 * lda + c0, lda * sizeof(double),
                           rows * sizeof(double), tm[j], hipMemcpyDeviceToHost, s) != hipSuccess)
        return false;
    }
    hipEvent_t e = evs.make();
    return e && hipEventRecord(e, s) == hipSuccess;
  };
  if (!download(0)) return fail(TLRQMC_EDEVICE, "copy of the factor failed");
  for (size_t g = 0; g < groups.size(); ++g) {
    const auto t_dl = clk::now();
    if (hipEventSynchronize(evs.evs[g]) != hipSuccess) return fail(TLRQMC_EDEVICE, "copy of the factor failed");
    if (g + 1 < groups.size() && !download(g + 1)) return fail(TLRQMC_EDEVICE, "copy of the factor failed");
    const auto t_cp = clk::now();
    phase[1] += secs(t_dl, t_cp);
    const int j0 = groups[g].first, j1 = groups[g].second;
    const double *src = stage[g % 2];
    std::vector<std::pair<int, int>> tiles;
    for (int j = j0; j < j1; ++j) {
      const int64_t rows = n - static_cast<int64_t>(j) * m;
      const double *panel = src + (poff[j] - poff[j0]);
      for (int t = 0; t < tm[j]; ++t)
        for (int u = 0; u < tm[j]; ++u)
          hdiag[doff[j] + static_cast<int64_t>(t) * tm[j] + u] = u <= t ? panel[static_cast<size_t>(u) * rows + t] : 0.0;
      for (int i = j + 1; i < r; ++i) tiles.push_back({i, j});
    }
    int hits = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : hits)
    for (size_t q = 0; q < tiles.size(); ++q) {
      const int i = tiles[q].first, j = tiles[q].second;
      const int64_t c0 = static_cast<int64_t>(j) * m, rows = n - c0;
      const double *T = src + (poff[j] - poff[j0]) + (static_cast<int64_t>(i) * m - c0);
      bool capped = false;
      const int k = compress_tile(T, rows, tm[i], tm[j], tol, max_rank, Us[static_cast<size_t>(i) * r + j],
                                  Vs[static_cast<size_t>(i) * r + j], capped);
      ranks[static_cast<size_t>(i) * r + j] = k;
      hits += capped ? 1 : 0;
    }
    cap_hits += hits;
    phase[2] += secs(t_cp, clk::now());
  }
  Aguard.reset();
  const auto t_layout = clk::now();
  std::vector<double> hU, hV;
  for (int i = 1; i < r; ++i)
    for (int j = 0; j < i; ++j) {
      const auto &u = Us[static_cast<size_t>(i) * r + j];
      const auto &v = Vs[static_cast<size_t>(i) * r + j];
      hU.insert(hU.end(), u.begin(), u.end());
      hV.insert(hV.end(), v.begin(), v.end());
    }
  st = factor_build(ctx, n, m, p.data(), hdiag.data(), ranks.data(), hU.data(), hV.data(), cap_hits, out);
  if (st) return st;
  phase[3] = secs(t_layout, clk::now());
  for (int k = 0; k < 4; ++k) (*out)->setup_seconds[k] = phase[k];
  (*out)->host_tiles = static_cast<int64_t>(r) * (r - 1) / 2;
  return cap_hits > 0 ? TLRQMC_WARN_RANKCAP : TLRQMC_OK;
}

// Block reordering during the Cholesky factorization of A (lower part,
// order p, limits al, bl in that order): on return A holds the factor and p,
// al, bl the final order (al, bl conditioned).
int rbodr_eliminate(tlrqmc_ctx *ctx, rocblas_handle h, double *A, int64_t lda, int64_t n, int m,
                    std::vector<int32_t> &p, std::vector<double> &al, std::vector<double> &bl) {
  hipStream_t s = ctx->stream;
  int st;
  const int r = static_cast<int>((n + m - 1) / m);
  const int nsort = (n % m == 0) ? r : r - 1;  // a ragged last block stays last
  // device work buffers
  Scratch sc(ctx);
  const int64_t mm = static_cast<int64_t>(m) * m;
  double *d_pack = sc.get<double>(static_cast<size_t>(std::max(nsort, 1)) * mm);
  double *d_tmp = sc.get<double>(static_cast<size_t>(2) * m * n);
  int32_t *d_idx = sc.get<int32_t>(static_cast<size_t>(2) * m + 2 * n);
  double *d_y = sc.get<double>(m);
  double *d_t = sc.get<double>(n);
  if (!d_pack || !d_tmp || !d_idx || !d_y || !d_t) return fail(TLRQMC_ENOMEM, "device allocation failed");
  int32_t *d_rows = d_idx, *d_src = d_idx + 2 * m, *d_slot = d_src + n;
  double *h_pack = ctx->pinned(3, static_cast<size_t>(std::max(nsort, 1)) * mm * sizeof(double));
  if (!h_pack) return fail(TLRQMC_ENOMEM, "pinned host allocation failed");
  std::vector<int32_t> src(n), slot(n, -1), rows;
  std::iota(src.begin(), src.end(), 0);
  std::vector<double> tvec(n);
  auto sym_block = [&](const double *blk, int mb, std::vector<double> &S) {
    S.resize(static_cast<size_t>(mb) * mb);
    for (int u = 0; u < mb; ++u)
      for (int v = 0; v < mb; ++v) S[static_cast<size_t>(u) * mb + v] = blk[static_cast<size_t>(v) * m + u];
  };
  for (int j = 0; j < r; ++j) {
    const int64_t j0 = static_cast<int64_t>(j) * m;
    const int mj = static_cast<int>(std::min<int64_t>(m, n - j0));
    // score the remaining full blocks on the current conditional problem
    const int cnt = j < nsort ? nsort - j : 1;
    const int mb_last = j < nsort ? m : mj;
    {
      SharedDevice dev;
      launch_pack_diag(s, A, lda, j0, m, mb_last, cnt, d_pack);
      if (hipMemcpyAsync(h_pack, d_pack, static_cast<size_t>(cnt) * mm * sizeof(double), hipMemcpyDeviceToHost,
                         s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return fail(TLRQMC_EDEVICE, "copy of the diagonal blocks failed");
    }
    std::vector<double> score(cnt);
    std::vector<std::vector<int>> order(cnt);
    std::vector<std::vector<double>> ymean(cnt);
#pragma omp parallel for schedule(dynamic, 1)
    for (int l = 0; l < cnt; ++l) {
      std::vector<double> S, la(al.begin() + j0 + static_cast<int64_t>(l) * m,
                                al.begin() + j0 + static_cast<int64_t>(l) * m + mb_last),
          lb(bl.begin() + j0 + static_cast<int64_t>(l) * m, bl.begin() + j0 + static_cast<int64_t>(l) * m + mb_last);
      sym_block(h_pack + static_cast<int64_t>(l) * mm, mb_last, S);
      score[l] = univariate_conditioning(mb_last, S, la, lb, order[l], &ymean[l]);
    }
    int t = 0;
    for (int l = 1; l < cnt; ++l)
      if (score[l] < score[t]) t = l;
    // positions j0.. take the chosen block (in its univariate-conditioning
    // order) first; the block it displaces moves to the chosen one's place
    rows.clear();
    for (int u = 0; u < mj; ++u) {
      src[j0 + u] = static_cast<int32_t>(j0 + static_cast<int64_t>(t) * m + order[t][u]);
      rows.push_back(static_cast<int32_t>(j0 + u));
    }
    if (t != 0)
      for (int u = 0; u < m; ++u) {
        const int64_t q = j0 + static_cast<int64_t>(t) * m + u;
        src[q] = static_cast<int32_t>(j0 + u);
        rows.push_back(static_cast<int32_t>(q));
      }
    bool moved = false;
    for (int32_t q : rows) moved = moved || src[q] != q;
    if (moved) {
      for (size_t k = 0; k < rows.size(); ++k) slot[rows[k]] = static_cast<int32_t>(k);
      if (hipMemcpyAsync(d_rows, rows.data(), rows.size() * sizeof(int32_t), hipMemcpyHostToDevice, s) != hipSuccess ||
          hipMemcpyAsync(d_src, src.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, s) != hipSuccess ||
          hipMemcpyAsync(d_slot, slot.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(TLRQMC_EDEVICE, "copy of the reordering failed");
      {
        SharedDevice dev;
        launch_permute_rows(s, A, lda, n, j0, static_cast<int>(rows.size()), d_rows, d_src, d_slot, d_tmp);
        if (hipStreamSynchronize(s) != hipSuccess) return fail(TLRQMC_EDEVICE, "reordering kernel failed");
      }
      std::vector<int32_t> np(rows.size());
      std::vector<double> na(rows.size()), nb(rows.size());
      for (size_t k = 0; k < rows.size(); ++k) {
        np[k] = p[src[rows[k]]];
        na[k] = al[src[rows[k]]];
        nb[k] = bl[src[rows[k]]];
      }
      for (size_t k = 0; k < rows.size(); ++k) {
        p[rows[k]] = np[k];
        al[rows[k]] = na[k];
        bl[rows[k]] = nb[k];
      }
      for (int32_t q : rows) {
        src[q] = q;
        slot[q] = -1;
      }
    }
    // factor the block, solve the panel below, condition the later limits
    // on the block's truncated means, update the Schur complement
    double *Ajj = A + j0 * lda + j0;
    if ((st = device_potrf(ctx, mj, Ajj, lda, j0, m))) return st;
    const int64_t rest = n - j0 - mj;
    if (rest > 0) {
      const double one = 1.0, zero = 0.0, minus = -1.0;
      double *P = Ajj + mj;
      if (hipMemcpyAsync(d_y, ymean[t].data(), mj * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(TLRQMC_EDEVICE, "copy failed");
      ExclusiveDevice dev;
      if (!dev.ok) return fail(TLRQMC_EDEVICE, "device synchronize failed");
      if (rocblas_dtrsm(h, rocblas_side_right, rocblas_fill_lower, rocblas_operation_transpose,
                        rocblas_diagonal_non_unit, static_cast<rocblas_int>(rest), mj, &one, Ajj,
                        static_cast<rocblas_int>(lda), P, static_cast<rocblas_int>(lda)) != rocblas_status_success ||
          rocblas_dgemv(h, rocblas_operation_none, static_cast<rocblas_int>(rest), mj, &one, P,
                        static_cast<rocblas_int>(lda), d_y, 1, &zero, d_t, 1) != rocblas_status_success ||
          rocblas_dsyrk(h, rocblas_fill_lower, rocblas_operation_none, static_cast<rocblas_int>(rest), mj, &minus, P,
                        static_cast<rocblas_int>(lda), &one, Ajj + mj * lda + mj,
                        static_cast<rocblas_int>(lda)) != rocblas_status_success)
        return fail(TLRQMC_EDEVICE, "rocBLAS update failed");
      if (hipMemcpyAsync(tvec.data(), d_t, rest * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return fail(TLRQMC_EDEVICE, "copy of the limit update failed");
      for (int64_t i = 0; i < rest; ++i) {
        al[j0 + mj + i] -= tvec[i];
        bl[j0 + mj + i] -= tvec[i];
      }
    }
  }
  return TLRQMC_OK;
}

}  // namespace

void DeviceLock::lock_shared() {
  std::unique_lock<std::mutex> l(mu_);
  cv_.wait(l, [&] { return !writer_ && writers_waiting_ == 0; });
  ++readers_;
}

void DeviceLock::unlock_shared() {
  std::lock_guard<std::mutex> l(mu_);
  if (--readers_ == 0) cv_.notify_all();
}

void DeviceLock::lock() {
  std::unique_lock<std::mutex> l(mu_);
  ++writers_waiting_;
  cv_.wait(l, [&] { return !writer_ && readers_ == 0; });
  --writers_waiting_;
  writer_ = true;
}

void DeviceLock::unlock() {
  std::lock_guard<std::mutex> l(mu_);
  writer_ = false;
  cv_.notify_all();
}

DeviceLock &device_lock() {
  static DeviceLock d;
  return d;
}

SharedDevice::SharedDevice() {
  if (t_shared_depth++ == 0) device_lock().lock_shared();
}

SharedDevice::~SharedDevice() {
  if (--t_shared_depth == 0) device_lock().unlock_shared();
}

ExclusiveDevice::ExclusiveDevice() {
  held_shared_ = t_shared_depth;
  if (held_shared_ > 0) {
    t_shared_depth = 0;
    device_lock().unlock_shared();
  }
  device_lock().lock();
  ok = hipDeviceSynchronize() == hipSuccess;
}

ExclusiveDevice::~ExclusiveDevice() {
  device_lock().unlock();
  if (held_shared_ > 0) {
    device_lock().lock_shared();
    t_shared_depth = held_shared_;
  }
}

rocblas_handle_t blas_handle(tlrqmc_ctx *ctx) { return blas_of(ctx); }

int device_cholesky(tlrqmc_ctx *ctx, double *A, int64_t lda, int64_t n) {
  return device_potrf(ctx, n, A, lda, 0, static_cast<int>(std::max<int64_t>(n, 1)));
}

int factor_from_device_dense(tlrqmc_ctx *ctx, int64_t n, const double *S, int64_t lds, const double *a,
                             const double *b, const double *xy, int m, double tol, int max_rank, int order,
                             int32_t *perm_out, tlrqmc_factor **out) {
  *out = nullptr;
  std::vector<int32_t> p(n);
  if (xy) morton(n, xy, p.data());
  else std::iota(p.begin(), p.end(), 0);
  double phase[4] = {0, 0, 0, 0};
  const auto t_begin = clk::now();
  hipStream_t s = ctx->stream;
  const int64_t lda = round_up(n, 64);
  double *A = static_cast<double *>(ctx->dmalloc(static_cast<size_t>(lda) * n * sizeof(double)));
  if (!A) return fail(TLRQMC_ENOMEM, "device allocation of the %lld x %lld covariance failed",
                      static_cast<long long>(n), static_cast<long long>(n));
  std::unique_ptr<double, std::function<void(double *)>> Aguard(A, [ctx](double *q) {
    (void)hipStreamSynchronize(ctx->stream);
    ctx->dfree(q);
  });
  int32_t *dp = static_cast<int32_t *>(ctx->dmalloc(n * sizeof(int32_t)));
  if (!dp) return fail(TLRQMC_ENOMEM, "device allocation failed");
  std::unique_ptr<int32_t, std::function<void(int32_t *)>> pguard(dp, [ctx](int32_t *q) {
    (void)hipStreamSynchronize(ctx->stream);
    ctx->dfree(q);
  });
  if (hipMemcpyAsync(dp, p.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, s) != hipSuccess)
    return fail(TLRQMC_EDEVICE, "copy of the order failed");
  {
    SharedDevice dev;
    launch_gather_sym(s, S, lds, dp, A, lda, n);
    if (hipStreamSynchronize(s) != hipSuccess) return fail(TLRQMC_EDEVICE, "covariance gather failed");
  }
  rocblas_handle h = blas_of(ctx);
  if (!h) return fail(TLRQMC_EDEVICE, "rocblas_create_handle failed");
  int st;
  if (order == 2) {
    std::vector<double> al(n), bl(n);
    for (int64_t i = 0; i < n; ++i) {
      al[i] = a[p[i]];
      bl[i] = b[p[i]];
    }
    if ((st = rbodr_eliminate(ctx, h, A, lda, n, m, p, al, bl))) return st;
  } else {
    if ((st = device_potrf(ctx, n, A, lda, 0, m))) return st;
  }
  phase[0] = secs(t_begin, clk::now());
  if (perm_out) std::copy(p.begin(), p.end(), perm_out);
  return compress_build(ctx, A, lda, n, m, p, tol, max_rank, phase, Aguard, out);
}

}  // namespace tlrqmc

using namespace tlrqmc;

extern "C" {

int tlrqmc_geometric_order(int64_t n, const tlrqmc_cov *cov, int32_t *perm_out) {
  clear_error();
  if (n < 1 || !perm_out) return fail(TLRQMC_EINVAL, "n must be >= 1 and perm_out non-null");
  int st = check_cov(n, cov);
  if (st) return st;
  if (cov->kind == 1) morton(n, cov->xy, perm_out);
  else std::iota(perm_out, perm_out + n, 0);
  return TLRQMC_OK;
}

int block_reorder(tlrqmc_ctx *, int64_t n, const tlrqmc_cov *cov, const double *a, const double *b, int m,
                  int32_t *perm_out) {
  clear_error();
  if (n < 1 || m < 1 || !a || !b || !perm_out) return fail(TLRQMC_EINVAL, "bad arguments to block_reorder");
  int st = check_cov(n, cov);
  if (st) return st;
  for (int64_t i = 0; i < n; ++i)
    if (std::isnan(a[i]) || std::isnan(b[i])) return fail(TLRQMC_EINVAL, "NaN limit at variable %lld", static_cast<long long>(i));
  std::vector<int32_t> base(n);
  if (cov->kind == 1) morton(n, cov->xy, base.data());
  else std::iota(base.begin(), base.end(), 0);
  const int64_t nblk = (n + m - 1) / m;
  const int64_t nsort = (n % m == 0) ? nblk : nblk - 1;
  std::vector<std::vector<int32_t>> blocks(nblk);
  std::vector<double> score(nblk);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t q = 0; q < nblk; ++q) {
    const int64_t i0 = q * m;
    const int mb = static_cast<int>(std::min<int64_t>(m, n - i0));
    std::vector<double> S(static_cast<size_t>(mb) * mb), al(mb), bl(mb);
    for (int i = 0; i < mb; ++i) {
      al[i] = a[base[i0 + i]];
      bl[i] = b[base[i0 + i]];
      for (int j = 0; j < mb; ++j) S[static_cast<size_t>(i) * mb + j] = cov_entry(cov, base[i0 + i], base[i0 + j]);
    }
    std::vector<int> order;
    score[q] = univariate_conditioning(mb, S, al, bl, order);
    blocks[q].resize(mb);
    for (int i = 0; i < mb; ++i) blocks[q][i] = base[i0 + order[i]];
  }
  for (int64_t j = 0; j < nsort; ++j) {
    int64_t best = j;
    for (int64_t l = j + 1; l < nsort; ++l)
      if (score[l] < score[best]) best = l;
    if (best != j) {
      std::swap(score[j], score[best]);
      std::swap(blocks[j], blocks[best]);
    }
  }
  int64_t o = 0;
  for (auto &blk : blocks)
    for (int32_t v : blk) perm_out[o++] = v;
  return TLRQMC_OK;
}

int tlr_factor(tlrqmc_ctx *ctx, int64_t n, const tlrqmc_cov *cov, const int32_t *perm, int m, double tol,
               int max_rank, tlrqmc_factor **out) {
  clear_error();
  if (!ctx || !out) return fail(TLRQMC_EINVAL, "null context or output");
  *out = nullptr;
  if (n < 1 || m < 1) return fail(TLRQMC_EINVAL, "n and m must be >= 1");
  if (!(tol >= 0.0)) return fail(TLRQMC_EINVAL, "tol must be >= 0");
  if (max_rank < 0) return fail(TLRQMC_EINVAL, "max_rank must be >= 0");
  int st = check_cov(n, cov);
  if (st) return st;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(TLRQMC_EDEVICE, "hipSetDevice failed");
  std::vector<int32_t> p;
  if ((st = order_of(n, cov, perm, p))) return st;
  double phase[4] = {0, 0, 0, 0};
  const auto t_begin = clk::now();
  const int64_t lda = round_up(n, 64);
  double *A = static_cast<double *>(ctx->dmalloc(static_cast<size_t>(lda) * n * sizeof(double)));
  if (!A) return fail(TLRQMC_ENOMEM, "device allocation of the %lld x %lld covariance failed",
                      static_cast<long long>(n), static_cast<long long>(n));
  std::unique_ptr<double, std::function<void(double *)>> Aguard(A, [ctx](double *q) {
    (void)hipStreamSynchronize(ctx->stream);
    ctx->dfree(q);
  });
  if ((st = build_cov(ctx, n, cov, p, A, lda))) return st;
  rocblas_handle h = blas_of(ctx);
  if (!h) return fail(TLRQMC_EDEVICE, "rocblas_create_handle failed");
  if ((st = device_potrf(ctx, n, A, lda, 0, m))) return st;
  phase[0] = secs(t_begin, clk::now());
  return compress_build(ctx, A, lda, n, m, p, tol, max_rank, phase, Aguard, out);
}

int tlr_factor_rbodr(tlrqmc_ctx *ctx, int64_t n, const tlrqmc_cov *cov, const double *a, const double *b, int m,
                     double tol, int max_rank, int32_t *perm_out, tlrqmc_factor **out) {
  clear_error();
  if (!ctx || !out || !a || !b) return fail(TLRQMC_EINVAL, "null argument");
  *out = nullptr;
  if (n < 1 || m < 1) return fail(TLRQMC_EINVAL, "n and m must be >= 1");
  if (!(tol >= 0.0)) return fail(TLRQMC_EINVAL, "tol must be >= 0");
  if (max_rank < 0) return fail(TLRQMC_EINVAL, "max_rank must be >= 0");
  int st = check_cov(n, cov);
  if (st) return st;
  for (int64_t i = 0; i < n; ++i)
    if (std::isnan(a[i]) || std::isnan(b[i])) return fail(TLRQMC_EINVAL, "NaN limit at variable %lld", static_cast<long long>(i));
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(TLRQMC_EDEVICE, "hipSetDevice failed");
  std::vector<int32_t> p;
  if ((st = order_of(n, cov, nullptr, p))) return st;
  double phase[4] = {0, 0, 0, 0};
  const auto t_begin = clk::now();
  hipStream_t s = ctx->stream;
  const int64_t lda = round_up(n, 64);
  double *A = static_cast<double *>(ctx->dmalloc(static_cast<size_t>(lda) * n * sizeof(double)));
  if (!A) return fail(TLRQMC_ENOMEM, "device allocation of the %lld x %lld covariance failed",
                      static_cast<long long>(n), static_cast<long long>(n));
  std::unique_ptr<double, std::function<void(double *)>> Aguard(A, [ctx](double *q) {
    (void)hipStreamSynchronize(ctx->stream);
    ctx->dfree(q);
  });
  if ((st = build_cov(ctx, n, cov, p, A, lda))) return st;
  rocblas_handle h = blas_of(ctx);
  if (!h) return fail(TLRQMC_EDEVICE, "rocblas_create_handle failed");
  // limits in the working order (conditioned as the elimination proceeds)
  std::vector<double> al(n), bl(n);
  for (int64_t i = 0; i < n; ++i) {
    al[i] = a[p[i]];
    bl[i] = b[p[i]];
  }
  if ((st = rbodr_eliminate(ctx, h, A, lda, n, m, p, al, bl))) return st;
  phase[0] = secs(t_begin, clk::now());
  if (perm_out) std::copy(p.begin(), p.end(), perm_out);
  return compress_build(ctx, A, lda, n, m, p, tol, max_rank, phase, Aguard, out);
}

}  // extern "C"

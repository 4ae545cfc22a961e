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

// ------------------------------------------- block reordering during Cholesky
// The working matrix is symmetric and stored in its lower triangle
// (column-major, leading dimension lda); columns before j0 already hold
// factor columns.

__device__ __forceinline__ double sym_at(const double *A, int64_t lda, int64_t p, int64_t q) {
  return p >= q ? A[q * lda + p] : A[p * lda + q];
}

// Copy count diagonal blocks of size mb (mb <= m; blocks start every m
// positions from j0) into out: block l at out + l m^2, entry (u, v) at
// v m + u; lower triangles mirrored.
__global__ __launch_bounds__(256) void k_pack_diag(const double *A, int64_t lda, int64_t j0, int m, int mb,
                                                   double *out) {
  const int l = blockIdx.y;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (e >= static_cast<int64_t>(m) * m) return;
  const int u = static_cast<int>(e % m), v = static_cast<int>(e / m);
  if (u >= mb || v >= mb) return;
  const int64_t b0 = j0 + static_cast<int64_t>(l) * m;
  out[static_cast<int64_t>(l) * m * m + e] = sym_at(A, lda, b0 + u, b0 + v);
}

// Row rows[k] of the matrix, every column (factor part and symmetric part),
// into tmp + k n.
__global__ __launch_bounds__(256) void k_gather_rows(const double *A, int64_t lda, int64_t n, int64_t j0,
                                                     const int32_t *rows, double *tmp) {
  const int k = blockIdx.y;
  const int64_t c = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (c >= n) return;
  const int64_t r = rows[k];
  tmp[static_cast<int64_t>(k) * n + c] = c < j0 ? A[c * lda + r] : sym_at(A, lda, r, c);
}

// Writes the rows rows[k] of the reordered matrix: new(P, c) = old(src[P],
// src[c]) for the symmetric part (c >= j0) and old(src[P], c) for the factor
// part, reading old values only from tmp (row slot[src[P]] holds old row
// src[P]; slot maps a position in rows to its k, -1 elsewhere).
__global__ __launch_bounds__(256) void k_scatter_rows(double *A, int64_t lda, int64_t n, int64_t j0,
                                                      const int32_t *rows, const int32_t *src,
                                                      const int32_t *slot, const double *tmp) {
  const int k = blockIdx.y;
  const int64_t c = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (c >= n) return;
  const int64_t P = rows[k];
  const int64_t sp = src[P];
  const double *old_row = tmp + static_cast<int64_t>(slot[sp]) * n;
  if (c < j0) {
    A[c * lda + P] = old_row[c];
  } else {
    const double v = old_row[src[c]];
    if (P >= c) A[c * lda + P] = v;
    else A[P * lda + c] = v;
  }
}

// A(i, j) = S(p[i], p[j]) on the lower triangle (S symmetric, lower stored).
__global__ __launch_bounds__(256) void k_gather_sym(const double *S, int64_t lds, const int32_t *p, double *A,
                                                    int64_t lda, int64_t n, int64_t col0) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const int64_t j = col0 + blockIdx.y;
  if (i >= n || i < j) return;
  A[j * lda + i] = sym_at(S, lds, p[i], p[j]);
}

// Lower triangle of the identity.
__global__ __launch_bounds__(256) void k_set_identity(double *A, int64_t lda, int64_t n, int64_t col0) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const int64_t j = col0 + blockIdx.y;
  if (i >= n || i < j) return;
  A[j * lda + i] = i == j ? 1.0 : 0.0;
}

void launch_gather_sym(hipStream_t s, const double *S, int64_t lds, const int32_t *p, double *A, int64_t lda,
                       int64_t n) {
  for (int64_t c = 0; c < n; c += 65535) {
    const int64_t nc = n - c < 65535 ? n - c : 65535;
    hipLaunchKernelGGL(k_gather_sym, dim3(static_cast<unsigned>((n + 255) / 256), static_cast<unsigned>(nc)),
                       dim3(256), 0, s, S, lds, p, A, lda, n, c);
  }
}

void launch_set_identity(hipStream_t s, double *A, int64_t lda, int64_t n) {
  for (int64_t c = 0; c < n; c += 65535) {
    const int64_t nc = n - c < 65535 ? n - c : 65535;
    hipLaunchKernelGGL(k_set_identity, dim3(static_cast<unsigned>((n + 255) / 256), static_cast<unsigned>(nc)),
                       dim3(256), 0, s, A, lda, n, c);
  }
}

void launch_pack_diag(hipStream_t s, const double *A, int64_t lda, int64_t j0, int m, int mb, int count,
                      double *out) {
  const int64_t mm = static_cast<int64_t>(m) * m;
  hipLaunchKernelGGL(k_pack_diag, dim3(static_cast<unsigned>((mm + 255) / 256), static_cast<unsigned>(count)),
                     dim3(256), 0, s, A, lda, j0, m, mb, out);
}

void launch_permute_rows(hipStream_t s, double *A, int64_t lda, int64_t n, int64_t j0, int nrows,
                         const int32_t *rows, const int32_t *src, const int32_t *slot, double *tmp) {
  const dim3 grid(static_cast<unsigned>((n + 255) / 256), static_cast<unsigned>(nrows));
  hipLaunchKernelGGL(k_gather_rows, grid, dim3(256), 0, s, A, lda, n, j0, rows, tmp);
  hipLaunchKernelGGL(k_scatter_rows, grid, dim3(256), 0, s, A, lda, n, j0, rows, src, slot, tmp);
}

}  // namespace tlrqmc

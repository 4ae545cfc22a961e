// Dense Cholesky factorization A = L L^T (lower, in place, column-major with
// leading dimension lda) on the device, blocked on two levels: panels of 256
// columns, each factored as four 64-column steps
//   k_chol_diag  : the 64 x 64 diagonal block, in LDS (one work-group); it
//                  also writes a row-major copy of the block and the
//                  reciprocals of its diagonal to a small scratch buffer;
//   k_chol_trsm  : the column block below it, L21 = A21 L11^-T, one lane per
//                  row (the row in registers, L11 through scalar loads);
//   k_chol_syrk  : the update of the rest of the panel's columns by that
//                  block, on 64 x 64 tiles with FP64 matrix cores
//                  (v_mfma_f64_16x16x4_f64);
// then one update of the trailing matrix by the whole panel (k_chol_wide:
// 256 x 128 tiles, 256-deep products on the matrix cores), so the trailing
// matrix is read and written once per 256 columns.  All arithmetic is FP64;
// the upper triangle of A is not referenced.  The setup step of the
// estimator (Section 3.3: the Cholesky factor of the covariance, then
// tile-wise compression) runs on these kernels.
#include "device_math.hpp"
#include "internal.hpp"
#include "setup_kernels.hpp"

namespace tlrqmc {

using namespace dev;

namespace {

constexpr int CB = kCholBlock;
typedef double f64x4 __attribute__((ext_vector_type(4)));

// Diagonal block at (k0, k0), b = min(64, n - k0) rows.  Right-looking
// over its columns with the block in registers: thread t holds row
// i = t % 64 at the columns congruent to g = t / 64 modulo 4 (wave g owns
// those columns).  At column j the owning wave takes the pivot from lane j,
// forms L(:, j) and publishes it in LDS (two buffers, alternating); after
// one barrier every thread subtracts L(i, j) L(c, j) from each of its
// entries.  Entries above the diagonal also receive these updates but are
// never read or stored, and L(r, j) is published as zero for r <= j, so the
// update needs no predicate.  Each entry sees the same fma updates in the
// same order as an in-place factorization.  On a non-positive pivot the
// global row index + 1 goes to *info and every later block leaves at once.
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const uint64_t u = static_cast<uint64_t>(__double_as_longlong(v));
  const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(u & 0xffffffffu), lane));
  const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(u >> 32), lane));
  return __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(hi) << 32) | lo));
}

__global__ __launch_bounds__(256) void k_chol_diag(double *A, int64_t lda, int64_t n, int64_t k0, int32_t *info,
                                                   double *scratch) {
  __shared__ double col[2][CB];
  __shared__ int bad;
  if (*info != 0) return;  // an earlier block failed (the same for the whole group)
  const int t = static_cast<int>(threadIdx.x);
  const int i = t & (CB - 1), g = t >> 6;
  const int b = static_cast<int>(min<int64_t>(CB, n - k0));
  double *D = A + k0 * lda + k0;
  double r[CB / 4];
#pragma unroll
  for (int k = 0; k < CB / 4; ++k) {
    const int c = 4 * k + g;
    r[k] = (i < b && c <= i) ? D[c * lda + i] : 0.0;
  }
  if (t == 0) bad = 0;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    if (j >= b) break;  // uniform
    double *cj = col[j & 1];
    if (g == (j & 3)) {  // the wave that owns column j
      const double piv = readlane_f64(r[j >> 2], j);
      if (piv > 0.0) {
        const double d = sqrt(piv);
        const double l = i > j ? r[j >> 2] / d : (i == j ? d : 0.0);
        r[j >> 2] = l;
        cj[i] = i > j ? l : 0.0;
        if (i == j) scratch[CB * CB + j] = 1.0 / d;  // reciprocal diagonal for the panel solve
      } else if (i == 0) {
        bad = 1;
        *info = static_cast<int32_t>(k0 + j + 1);
      }
    }
    __syncthreads();
    if (bad) return;  // uniform: every thread reads the same flag after the barrier
    const double li = cj[i];
#pragma unroll
    for (int k = 0; k < CB / 4; ++k) r[k] = fma(-li, cj[4 * k + g], r[k]);
  }
#pragma unroll
  for (int k = 0; k < CB / 4; ++k) {
    const int c = 4 * k + g;
    if (i < b && c <= i) D[c * lda + i] = r[k];
    // row-major copy (row i of L11 contiguous) for the panel solve
    if (i < b) scratch[i * CB + c] = c <= i ? r[k] : 0.0;
  }
  if (g == 0 && i >= b) scratch[CB * CB + i] = 0.0;
}

// Panel rows r >= k0 + 64: x solves x L11^T = a, left-looking: step j
// loads a_j, forms x_j = (a_j - sum_{c<j} x_c L11(j, c)) / L11(j, j) and
// stores it, so a column's address lives only within its step.  The row of
// x stays in registers; row j of L11 comes from the row-major copy in the
// scratch buffer by scalar loads.
__global__ __launch_bounds__(256) void k_chol_trsm(double *A, int64_t lda, int64_t n, int64_t k0,
                                                   const double *scratch) {
  const int64_t r = k0 + CB + static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (r >= n) return;
  const auto Lr = as_const(scratch);  // Lr[j * 64 + c] = L11(j, c)
  const auto inv = as_const(scratch + CB * CB);
  const uint32_t ro = static_cast<uint32_t>(r);
  double x[CB];
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    double *col = A + (k0 + j) * lda;
    double acc = col[ro];
#pragma unroll
    for (int c = 0; c < j; ++c) acc = fma(-x[c], Lr[j * CB + c], acc);
    x[j] = acc * inv[j];
    col[ro] = x[j];
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Update of the lower tiles of A22 = A(k0+64:, k0+64:) in its first ntc
// tile columns: tile (ti, tj) = (blockIdx.x, blockIdx.y), ti >= tj, of 64 x
// 64; each of the four waves computes one 32 x 32 quarter as 2 x 2
// matrix-core tiles of 16 x 16 over the 64 columns of the block.  Operand
// layouts (as for the sweep's block products): A operand lane l = row l % 16,
// column 4 k + l / 16; B operand lane l = column l % 16 (a row of the panel),
// k-row 4 k + l / 16; the result lane l holds rows l / 16 + 4 r, column l % 16.
__global__ __launch_bounds__(256) void k_chol_syrk(double *A, int64_t lda, int64_t n, int64_t k0) {
  const int ti = static_cast<int>(blockIdx.x), tj = static_cast<int>(blockIdx.y);
  if (ti < tj) return;  // the whole group
  const int w = static_cast<int>(threadIdx.x) >> 6, l = static_cast<int>(threadIdx.x) & 63;
  const int64_t base = k0 + CB;
  const int64_t r0 = base + static_cast<int64_t>(ti) * CB + (w >> 1) * 32;
  const int64_t c0 = base + static_cast<int64_t>(tj) * CB + (w & 1) * 32;
  const auto P = as_global(A + k0 * lda);  // P[c * lda + row] = L21(row, c)
  f64x4 acc[2][2];
#pragma unroll
  for (int si = 0; si < 2; ++si)
#pragma unroll
    for (int sj = 0; sj < 2; ++sj) acc[si][sj] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ks = 0; ks < CB / 4; ++ks) {
    const int64_t col = static_cast<int64_t>(ks * 4 + (l >> 4)) * lda;
    double va[2], vb[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int64_t ra = r0 + s * 16 + (l & 15), rb = c0 + s * 16 + (l & 15);
      va[s] = ra < n ? P[col + ra] : 0.0;
      vb[s] = rb < n ? P[col + rb] : 0.0;
    }
#pragma unroll
    for (int si = 0; si < 2; ++si)
#pragma unroll
      for (int sj = 0; sj < 2; ++sj) acc[si][sj] = __builtin_amdgcn_mfma_f64_16x16x4f64(va[si], vb[sj], acc[si][sj], 0, 0, 0);
  }
#pragma unroll
  for (int si = 0; si < 2; ++si)
#pragma unroll
    for (int sj = 0; sj < 2; ++sj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + si * 16 + (l >> 4) + 4 * r, col = c0 + sj * 16 + (l & 15);
        if (row < n && col < n && row >= col) A[col * lda + row] -= acc[si][sj][r];
      }
}


// Trailing update A(k1:, k1:) -= P P^T with P = A(k1:, k0:k1), k1 = k0 + 256,
// on 256 x 128 tiles of the lower triangle with eight waves: the tiles of
// row block ti (256 rows) are the column blocks tj = 0 .. 2 ti + 1 (128
// columns), so tile b is (ti, b - ti (ti + 1)) with ti the largest t such
// that t (t + 1) <= b.  The two operand blocks of P (256 and 128 rows) go
// through LDS 16 columns at a time, double-buffered (the next chunk's global
// loads are in flight during the current chunk's products), stored k-major.
// Wave w computes the 64 x 64 block (w / 2, w % 2) as 4 x 4 matrix-core
// tiles (operand layouts as above); a wave whose block lies wholly above the
// diagonal loads and synchronises but computes nothing.
__global__ __launch_bounds__(512) void k_chol_wide(double *A, int64_t lda, int64_t n, int64_t k0) {
  constexpr int PW = kCholPanel, KC = 16, RA = 256, RB = 128;
  __shared__ double As[2][KC][RA + 4], Bs[2][KC][RB + 4];
  const int64_t tile = blockIdx.x;
  int64_t ti = static_cast<int64_t>((sqrt(4.0 * static_cast<double>(tile) + 1.0) - 1.0) * 0.5);
  while (ti * (ti + 1) > tile) --ti;
  while ((ti + 1) * (ti + 2) <= tile) ++ti;
  const int64_t tj = tile - ti * (ti + 1);
  const int t = static_cast<int>(threadIdx.x), w = t >> 6, l = t & 63;
  const int64_t base = k0 + PW;
  const int64_t ra0 = base + ti * RA, rb0 = base + tj * RB;
  const int64_t R0 = ra0 + (w >> 1) * 64, C0 = rb0 + (w & 1) * 64;
  const bool idle = R0 + 63 < C0;
  // loaders: A rows t % 256, columns t / 256 + 2 j (j < 8); B rows t % 128,
  // columns t / 128 + 4 j (j < 4)
  const int lra = t & (RA - 1), lca = t >> 8, lrb = t & (RB - 1), lcb = t >> 7;
  const bool oka = ra0 + lra < n, okb = rb0 + lrb < n;
  const uint32_t ua = oka ? static_cast<uint32_t>(ra0 + lra) : 0u;  // out-of-range rows read row 0, store zero
  const uint32_t ub = okb ? static_cast<uint32_t>(rb0 + lrb) : 0u;
  double ga[8], gb[4];
  auto gload = [&](int ch) {
#pragma unroll
    for (int j = 0; j < 8; ++j) ga[j] = as_global(A + (k0 + ch * KC + lca + 2 * j) * lda)[ua];
#pragma unroll
    for (int j = 0; j < 4; ++j) gb[j] = as_global(A + (k0 + ch * KC + lcb + 4 * j) * lda)[ub];
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int j = 0; j < 8; ++j) As[buf][lca + 2 * j][lra] = oka ? ga[j] : 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) Bs[buf][lcb + 4 * j][lrb] = okb ? gb[j] : 0.0;
  };
  f64x4 acc[4][4];
#pragma unroll
  for (int si = 0; si < 4; ++si)
#pragma unroll
    for (int sj = 0; sj < 4; ++sj) acc[si][sj] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int wa = (w >> 1) * 64 + (l & 15), wb = (w & 1) * 64 + (l & 15), kl = l >> 4;
  gload(0);
  sstore(0);
  __syncthreads();
#pragma unroll 1
  for (int ch = 0; ch < PW / KC; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < PW / KC) gload(ch + 1);
    if (!idle) {
#pragma unroll
      for (int kk = 0; kk < KC / 4; ++kk) {
        double va[4], vb[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          va[s] = As[buf][4 * kk + kl][wa + 16 * s];
          vb[s] = Bs[buf][4 * kk + kl][wb + 16 * s];
        }
#pragma unroll
        for (int si = 0; si < 4; ++si)
#pragma unroll
          for (int sj = 0; sj < 4; ++sj)
            acc[si][sj] = __builtin_amdgcn_mfma_f64_16x16x4f64(va[si], vb[sj], acc[si][sj], 0, 0, 0);
      }
    }
    if (ch + 1 < PW / KC) sstore(buf ^ 1);
    __syncthreads();
  }
  if (idle) return;
#pragma unroll
  for (int si = 0; si < 4; ++si)
#pragma unroll
    for (int sj = 0; sj < 4; ++sj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = R0 + si * 16 + (l >> 4) + 4 * r, col = C0 + sj * 16 + (l & 15);
        if (row < n && col < n && row >= col) A[col * lda + row] -= acc[si][sj][r];
      }
}

}  // namespace

void launch_cholesky(hipStream_t s, double *A, int64_t lda, int64_t n, int32_t *info, double *scratch) {
  for (int64_t K0 = 0; K0 < n; K0 += kCholPanel) {
    const int64_t K1 = std::min<int64_t>(n, K0 + kCholPanel);
    for (int64_t k0 = K0; k0 < K1; k0 += CB) {
      hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(256), 0, s, A, lda, n, k0, info, scratch);
      const int64_t rest = n - k0 - CB;
      if (rest <= 0) break;
      hipLaunchKernelGGL(k_chol_trsm, dim3(static_cast<unsigned>((rest + 255) / 256)), dim3(256), 0, s, A, lda, n, k0,
                         scratch);
      // the panel's remaining columns (all rows below them)
      const int64_t ntc = (K1 - (k0 + CB) + CB - 1) / CB;
      if (ntc > 0)
        hipLaunchKernelGGL(k_chol_syrk, dim3(static_cast<unsigned>((rest + CB - 1) / CB), static_cast<unsigned>(ntc)),
                           dim3(256), 0, s, A, lda, n, k0);
    }
    const int64_t rest = n - K1;
    if (rest > 0) {
      const int64_t nt = (rest + 255) / 256;
      hipLaunchKernelGGL(k_chol_wide, dim3(static_cast<unsigned>(nt * (nt + 1))), dim3(512), 0, s, A, lda, n, K0);
    }
  }
}

}  // namespace tlrqmc

// Low-rank limit update of the FP64 form on FP64 matrix cores.
//
// The products of the TLR recursion (Section 3.4, TLR QMC for MVN: the
// limit update U_ij (V_ij^T y_j)) are GEMMs over the samples with the same
// operand addressing (this file runs the limit update; the projection, whose
// row count, the panel width, is often small against 128, stays on the
// vector ALU in kernels.hip, which measured faster):
//   limit update : Delta_i = U_row(i) Z_row(i)   A(t, q) = U_row[q lda + t]
//   projection   : Z(:, j) = V_panel(j)^T Y_j     A(c, t) = V_panel[t lda + c]
// and B(k, s) = In[k ld + s] (Z rows or the tile's y), C(row, s) written to
// Out[row ld + s] (the projection maps its rows).  The operand rows are
// zero-padded to lda (a multiple of 64).
//
// A work-group computes 128 rows x 128 samples; the two 128-wide operand
// blocks go through LDS 16 k at a time, double-buffered (the next chunk's
// global loads are in flight during the current chunk's products), stored
// k-major.  Wave w computes the 64 x 64 block (w / 2, w % 2) as 4 x 4 tiles
// of v_mfma_f64_16x16x4_f64 (A operand lane l = row l % 16, k l / 16; B
// operand lane l = sample l % 16, k l / 16; result lane l holds rows
// l / 16 + 4 r, sample l % 16).  All arithmetic is FP64.
#include <hip/hip_ext.h>

#include "device_math.hpp"
#include "internal.hpp"

namespace tlrqmc {

using namespace dev;

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int KC = 16, TR = kLr64Tile, LP = TR + 4;

__device__ __forceinline__ void lr64_body(const LrParams &p, int rb, int64_t sb) {
  __shared__ double As[2][KC][LP], Bs[2][KC][LP];
  const int t = static_cast<int>(threadIdx.x), w = t >> 6, l = t & 63;
  const int r0 = rb * TR;
  const int64_t s0 = sb * TR;
  // loader: thread t moves operand row t % 128 of k = t / 128 + 2 j, j < 8
  const int lr = t & (TR - 1), lc = t >> 7;
  const bool oka = r0 + lr < p.lda, okb = s0 + lr < p.count;
  const uint32_t ua = oka ? static_cast<uint32_t>(r0 + lr) : 0u;  // out of range: read index 0, store zero
  const int64_t ub = okb ? s0 + lr : 0;
  const double *Ap = p.Mat, *Bp = p.In;
  double ga[KC / 2], gb[KC / 2];
  auto gload = [&](int ch) {
#pragma unroll
    for (int j = 0; j < KC / 2; ++j) {
      const int k = ch * KC + lc + 2 * j;
      const bool kin = k < p.K;
      const int kk = kin ? k : 0;
      const double x = as_global(Ap + static_cast<int64_t>(kk) * p.lda)[ua];
      const double y = as_global(Bp + static_cast<int64_t>(kk) * p.ld)[ub];
      ga[j] = kin ? x : 0.0;
      gb[j] = kin ? y : 0.0;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int j = 0; j < KC / 2; ++j) {
      As[buf][lc + 2 * j][lr] = oka ? ga[j] : 0.0;
      Bs[buf][lc + 2 * j][lr] = okb ? gb[j] : 0.0;
    }
  };
  f64x4 acc[4][4];
#pragma unroll
  for (int si = 0; si < 4; ++si)
#pragma unroll
    for (int sj = 0; sj < 4; ++sj) acc[si][sj] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int wa = (w >> 1) * 64 + (l & 15), wb = (w & 1) * 64 + (l & 15), kl = l >> 4;
  const int nch = p.K > 0 ? (p.K + KC - 1) / KC : 0;  // K = 0: no loads, C = 0
  if (nch > 0) {
    gload(0);
    sstore(0);
  }
  __syncthreads();
#pragma unroll 1
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nch) gload(ch + 1);
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
    if (ch + 1 < nch) sstore(buf ^ 1);
    __syncthreads();
  }
  const int rw = r0 + (w >> 1) * 64;
  const int64_t sw = s0 + (w & 1) * 64;
#pragma unroll
  for (int si = 0; si < 4; ++si)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = rw + si * 16 + (l >> 4) + 4 * r;
      if (row >= p.rows) continue;
      double *o = p.Out + static_cast<int64_t>(row) * p.ld;
#pragma unroll
      for (int sj = 0; sj < 4; ++sj) {
        const int64_t s = sw + sj * 16 + (l & 15);
        if (s < p.count) o[s] = acc[si][sj][r];
      }
    }
}

__global__ __launch_bounds__(256) void k_lr64(LrParams p) {
  lr64_body(p, static_cast<int>(blockIdx.y), blockIdx.x);
}

// Batched: descriptor blockIdx.z; a block beyond its descriptor's extent
// leaves before any barrier (the condition is uniform over the block).
__global__ __launch_bounds__(256) void k_lr64_batch(const LrParams *ps) {
  const LrParams p = load_uniform(ps + blockIdx.z);
  if (static_cast<int64_t>(blockIdx.x) * TR >= p.count || static_cast<int>(blockIdx.y) * TR >= p.rows) return;
  lr64_body(p, static_cast<int>(blockIdx.y), blockIdx.x);
}


}  // namespace

void launch_delta_f64(hipStream_t s, const LrParams &p, const LaunchEvents &ev) {
  if (p.count <= 0 || p.rows <= 0) return;
  const Grid g = lr64_grid(p.count, p.rows, 1);
  hipExtLaunchKernelGGL(k_lr64, dim3(g.x, g.y, g.z), dim3(256), 0, s, ev.start, ev.stop, 0, p);
}

void launch_delta_f64_batch(hipStream_t s, const LrParams *d, int n, int64_t max_count, int max_rows) {
  if (n <= 0 || max_count <= 0 || max_rows <= 0) return;
  const Grid g = lr64_batch_grid(n, max_count, max_rows);
  hipLaunchKernelGGL(k_lr64_batch, dim3(g.x, g.y, g.z), dim3(256), 0, s, d);
}

}  // namespace tlrqmc

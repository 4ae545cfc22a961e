// Low-rank limit updates of the precision form on BF16 matrix cores.
//
// Both products of the TLR recursion (Section 3.4, TLR QMC for MVN: the
// limit update U_ij (V_ij^T y_j)) run as GEMMs over the samples:
//   k_delta_mfma : Delta_i = U_row(i) Z_row(i)     (m_i x K_row) (K_row x S)
//   k_zproj_mfma : Z(:, j) = V_panel(j)^T Y_j      (K_col x m_j) (m_j x S)
// Operands are split x = hi + lo into two BF16 numbers and multiplied as
// hi*hi + hi*lo + lo*hi (the lo*lo term, below 2^-16 relative, is dropped)
// with FP32 accumulation in v_mfma_f32_16x16x32_bf16.  The factor's U and V
// are split once when the factor is built; Z (FP32) and Y (FP64) are split
// when they are staged into LDS.
//
// Operand layout of v_mfma_f32_16x16x32_bf16 (checked on the device): lane
// l holds A[l % 16][8 (l / 16) + e] and B[8 (l / 16) + e][l % 16], e = 0..7,
// and receives C[4 (l / 16) + i][l % 16], i = 0..3.
#include "internal.hpp"

namespace tlrqmc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

// Round-to-nearest-even float -> bf16 bits (finite input).
__device__ __forceinline__ unsigned short bf16_bits(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<unsigned short>(u >> 16);
}

__device__ __forceinline__ void split2(float x, unsigned short &hi, unsigned short &lo) {
  hi = bf16_bits(x);
  lo = bf16_bits(x - __uint_as_float(static_cast<unsigned>(hi) << 16));
}

__device__ __forceinline__ f32x4 mfma3(u16x8 ah, u16x8 al, u16x8 bh, u16x8 bl, f32x4 c) {
  const bf16x8 AH = __builtin_bit_cast(bf16x8, ah), AL = __builtin_bit_cast(bf16x8, al);
  const bf16x8 BH = __builtin_bit_cast(bf16x8, bh), BL = __builtin_bit_cast(bf16x8, bl);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AL, BH, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AH, BL, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AH, BH, c, 0, 0, 0);
  return c;
}

}  // namespace

// Delta(r, s) = sum_k U(r, k) Z(k, s).  Block: 64 samples, 64 RT rows (four
// waves of RT row tiles); Z is staged per 32-deep k step in LDS, already in
// B-operand layout; U (row-major, k padded to 32, rows padded to 64 RT) is
// read straight from global memory in A-operand layout.
template <int RT>
__global__ __launch_bounds__(256) void k_delta_mfma(MfmaDeltaParams p) {
  __shared__ u16x8 Bs[2][4][64];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t s0 = static_cast<int64_t>(blockIdx.x) * 64;
  const int r0 = blockIdx.y * 64 * RT + w * 16 * RT;
  f32x4 acc[RT][4];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // staging role of this thread: sample tile st, B lane L
  const int st = threadIdx.x >> 6, L = threadIdx.x & 63;
  const int64_t ss = s0 + 16 * st + (L & 15);
  const bool sok = ss < p.count;
  for (int kk = 0; kk < p.KP; kk += 32) {
    u16x8 h, lo;
    const float *zc = p.Z + static_cast<int64_t>(kk + 8 * (L >> 4)) * p.ld + ss;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float z = (sok && kk + 8 * (L >> 4) + e < p.K) ? zc[static_cast<int64_t>(e) * p.ld] : 0.f;
      unsigned short a, b;
      split2(z, a, b);
      h[e] = a;
      lo[e] = b;
    }
    Bs[0][st][L] = h;
    Bs[1][st][L] = lo;
    __syncthreads();
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const int64_t ro = static_cast<int64_t>(r0 + 16 * rt + (l & 15)) * p.KP + kk + 8 * (l >> 4);
      const u16x8 ah = *reinterpret_cast<const u16x8 *>(p.Uhi + ro);
      const u16x8 al = *reinterpret_cast<const u16x8 *>(p.Ulo + ro);
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[rt][t] = mfma3(ah, al, Bs[0][t][l], Bs[1][t][l], acc[rt][t]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t s = s0 + 16 * t + (l & 15);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = r0 + 16 * rt + 4 * (l >> 4) + i;
        if (row < p.rows && s < p.count) p.Delta[static_cast<int64_t>(row) * p.ld + s] = acc[rt][t][i];
      }
    }
}

// Z(map(c), s) = sum_t V(t, c) Y(t, s).  Block: 64 samples; the whole Y
// tile (m_j rows, FP64) is split into BF16 hi/lo and kept in LDS in
// B-operand layout; the four waves then take 32-row passes over the K_col
// outputs, reading V^T (row-major, t padded to 32) from global memory.
__global__ __launch_bounds__(256) void k_zproj_mfma(MfmaZprojParams p) {
  extern __shared__ u16x8 Ys[];  // [mp/32][2][4][64]
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t s0 = static_cast<int64_t>(blockIdx.x) * 64;
  const int st = threadIdx.x >> 6, L = threadIdx.x & 63;
  const int64_t ss = s0 + 16 * st + (L & 15);
  const bool sok = ss < p.count;
  const int nk = p.mp >> 5;
  for (int kk = 0; kk < nk; ++kk) {
    u16x8 h, lo;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int t = 32 * kk + 8 * (L >> 4) + e;
      const float y = (sok && t < p.mj) ? static_cast<float>(p.Y[static_cast<int64_t>(t) * p.ld + ss]) : 0.f;
      unsigned short a, b;
      split2(y, a, b);
      h[e] = a;
      lo[e] = b;
    }
    Ys[((kk * 2 + 0) * 4 + st) * 64 + L] = h;
    Ys[((kk * 2 + 1) * 4 + st) * 64 + L] = lo;
  }
  __syncthreads();
  for (int pass = w; 32 * pass < p.Kc; pass += 4) {
    const int c0 = 32 * pass;
    f32x4 acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int kk = 0; kk < nk; ++kk) {
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
        const int64_t ro = static_cast<int64_t>(c0 + 16 * rt + (l & 15)) * p.mp + 32 * kk + 8 * (l >> 4);
        const u16x8 ah = *reinterpret_cast<const u16x8 *>(p.Vhi + ro);
        const u16x8 al = *reinterpret_cast<const u16x8 *>(p.Vlo + ro);
#pragma unroll
        for (int t = 0; t < 4; ++t)
          acc[rt][t] = mfma3(ah, al, Ys[((kk * 2 + 0) * 4 + t) * 64 + l], Ys[((kk * 2 + 1) * 4 + t) * 64 + l],
                             acc[rt][t]);
      }
    }
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t s = s0 + 16 * t + (l & 15);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int c = c0 + 16 * rt + 4 * (l >> 4) + i;
          if (c < p.Kc && s < p.count) p.Z[static_cast<int64_t>(p.map[c]) * p.ld + s] = acc[rt][t][i];
        }
      }
  }
}

int delta_mfma_rt(int rows) { return rows <= 64 ? 1 : rows <= 128 ? 2 : 4; }

void launch_delta_mfma(hipStream_t s, const MfmaDeltaParams &p) {
  const int rt = delta_mfma_rt(p.rows);
  const dim3 grid(static_cast<unsigned>((p.count + 63) / 64), static_cast<unsigned>((p.rows + 64 * rt - 1) / (64 * rt)));
  if (rt == 1) hipLaunchKernelGGL(k_delta_mfma<1>, grid, dim3(256), 0, s, p);
  else if (rt == 2) hipLaunchKernelGGL(k_delta_mfma<2>, grid, dim3(256), 0, s, p);
  else hipLaunchKernelGGL(k_delta_mfma<4>, grid, dim3(256), 0, s, p);
}

void launch_zproj_mfma(hipStream_t s, const MfmaZprojParams &p) {
  const size_t lds = static_cast<size_t>(p.mp / 32) * 2 * 4 * 64 * sizeof(u16x8);
  (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_zproj_mfma),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  hipLaunchKernelGGL(k_zproj_mfma, dim3(static_cast<unsigned>((p.count + 63) / 64)), dim3(256), lds, s, p);
}

}  // namespace tlrqmc

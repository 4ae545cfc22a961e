// Low-rank limit updates of the precision form on BF16 matrix cores.
//
// Both products of the TLR recursion (Section 3.4, TLR QMC for MVN: the
// limit update U_ij (V_ij^T y_j)) run as GEMMs over the samples, in one
// kernel template:
//   limit update : Delta_i = U_row(i) Z_row(i)     (m_i x K_row) (K_row x S)
//   projection   : Z(:, j) = V_panel(j)^T Y_j      (K_col x m_j) (m_j x S)
// Operands are split x = hi + lo into two BF16 numbers (each rounded to
// nearest even) and multiplied as
// hi*hi + hi*lo + lo*hi (the lo*lo term, below 2^-16 relative, is dropped)
// with FP32 accumulation in v_mfma_f32_16x16x32_bf16.  The factor's U and V
// are split once when the factor is built; Z (FP32) and Y (FP64) are split
// when they are staged into LDS.
//
// Operand layout of v_mfma_f32_16x16x32_bf16 (checked on the device): lane
// l holds A[l % 16][8 (l / 16) + e] and B[8 (l / 16) + e][l % 16], e = 0..7,
// and receives C[4 (l / 16) + i][l % 16], i = 0..3.
#include <hip/hip_ext.h>

#include <type_traits>

#include "device_math.hpp"
#include "internal.hpp"

namespace tlrqmc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// Split of eight values x = hi + lo into BF16 pairs, rounded to nearest even
// (v_cvt_pk_bf16_f32 two at a time); lo is the rounding error of hi, itself
// rounded, so hi + lo carries about 16 significant bits.
template <class TB>
__device__ __forceinline__ void split8(const TB (&v)[8], u16x8 &h, u16x8 &lo) {
  unsigned hw[4], lw[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const f32x2 x = {static_cast<float>(v[2 * e]), static_cast<float>(v[2 * e + 1])};
    const bf16x2 hb = __builtin_convertvector(x, bf16x2);
    const bf16x2 lb = __builtin_convertvector(x - __builtin_convertvector(hb, f32x2), bf16x2);
    hw[e] = __builtin_bit_cast(unsigned, hb);
    lw[e] = __builtin_bit_cast(unsigned, lb);
  }
  h = __builtin_bit_cast(u16x8, hw);
  lo = __builtin_bit_cast(u16x8, lw);
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

// C(row, s) = sum_k A(row, k) B(k, s).  Block: 16 NT samples and 64 RT
// rows (four waves of RT row tiles of 16; each wave covers all NT sample
// tiles).  B is staged per 32-deep k step in LDS, already split and in
// B-operand layout, double-buffered (wave w stages sample tiles w, w + 4,
// ...); the global loads of step k + 64 are issued before the matrix
// products of step k, so two steps of products cover their latency.  A
// (row-major, padded) is read straight from global memory one step ahead
// (it is small and shared by every sample block, so it stays in L2): a
// wider sample block divides its reads by NT / 4.
//
// The grid is one-dimensional.  Work-groups are dealt to the eight XCDs
// round robin, and each XCD has its own L2, so the linear id is remapped
// such that every XCD receives a contiguous range of (sample block, row
// block) pairs, row block fastest: the row blocks that share one sample
// block's B run back to back on one XCD and re-read B from its L2.
template <int RT, int NT, bool BD, bool MAP>
__device__ __forceinline__ void lr_mfma_body(const MfmaLrParams &p, unsigned bid, unsigned total) {
  static_assert(NT % 4 == 0, "four waves stage the sample tiles");
  constexpr int NS = NT / 4;  // sample tiles staged per wave
  __shared__ u16x8 Bs[2][2][NT][64];  // [buffer][hi, lo][sample tile][lane]
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int nrb = (p.rows + 64 * RT - 1) / (64 * RT);
  const unsigned q = total / 8, rm = total % 8;
  const unsigned xcd = bid % 8, idx = bid / 8;
  const unsigned logical = xcd * q + min(xcd, rm) + idx;
  // wave-uniform by construction; readfirstlane lets the compiler keep them
  // (and the buffer resources built from them) in scalar registers
  const unsigned rb = __builtin_amdgcn_readfirstlane(logical % static_cast<unsigned>(nrb));
  const unsigned sb = __builtin_amdgcn_readfirstlane(logical / static_cast<unsigned>(nrb));
  const int64_t s0 = static_cast<int64_t>(sb) * (16 * NT);
  const int r0 = static_cast<int>(rb) * 64 * RT + w * 16 * RT;
  f32x4 acc[RT][NT];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // staging role of this thread: sample tiles w + 4 u (u < NS), B lane l
  const int kq = 8 * (l >> 4);
  using TB = typename std::conditional<BD, double, float>::type;
  const TB *B = BD ? reinterpret_cast<const TB *>(p.Bd) : reinterpret_cast<const TB *>(p.Bf);
  static_assert(16 * NT <= 256, "sample blocks must divide the leading dimension's multiple of 256");
  // B through a buffer resource over the valid rows [kk, min(kk + 32, K))
  // of each step: a k past K lies past the resource and reads zero in
  // hardware, so no load is predicated or followed by a select (either
  // would make the wave wait for the load at once).  A lane past the
  // samples reads a column inside the leading dimension whose products land
  // only in outputs that are not stored.  Offsets are 32-bit: 32 ld
  // elements must stay below 2 GiB (the drivers bound ld).
  const uint32_t lane_off = static_cast<uint32_t>(kq * p.ld + 16 * w + (l & 15)) * sizeof(TB);
  const uint32_t row_bytes = static_cast<uint32_t>(p.ld * sizeof(TB));
  auto load_b = [&](int kk, TB (&v)[NS][8]) {
    // rows of this step (none past K: every load reads zero); readfirstlane
    // keeps the resource scalar (the clamp would otherwise go to the VALU)
    const int bytes = __builtin_amdgcn_readfirstlane(static_cast<int>(max(0, min(32, p.K - kk)) * row_bytes));
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<TB *>(B) + static_cast<int64_t>(kk) * p.ld + s0, 0, bytes, dev::kRawBufferWord3);
#pragma unroll
    for (int u = 0; u < NS; ++u)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int off = static_cast<int>(lane_off + (64 * u) * sizeof(TB) + e * row_bytes);
        if constexpr (BD) {
          v[u][e] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
        } else {
          v[u][e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
        }
      }
  };
  // A operand of one 32-deep step (this wave's row tiles), from global
  // memory.  A step past the end reads the last step's columns again: they
  // meet B rows of zero, so their products add exactly zero.
  auto load_a = [&](int kk, u16x8 (&ah)[RT], u16x8 (&al)[RT]) {
    const int kc = min(kk, p.KP - 32);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const int64_t ro = static_cast<int64_t>(r0 + 16 * rt + (l & 15)) * p.KP + kc + kq;
      ah[rt] = *reinterpret_cast<const u16x8 *>(p.Ahi + ro);
      al[rt] = *reinterpret_cast<const u16x8 *>(p.Alo + ro);
    }
  };
  // One 32-deep step: stage the B registers of this step into LDS buffer
  // buf, refill them with the step two ahead, fetch the next step's A
  // operand, multiply with this step's A.  The prefetches are issued
  // unconditionally (past the end they read zeros or repeat the last
  // columns): a conditional load would make the compiler wait for every
  // load in flight where the paths join.
  auto step = [&](int kk, TB (&v)[NS][8], int buf, u16x8 (&ah)[RT], u16x8 (&al)[RT], u16x8 (&nh)[RT],
                  u16x8 (&nl)[RT]) {
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      u16x8 h, lo;
      split8(v[u], h, lo);
      Bs[buf][0][w + 4 * u][l] = h;
      Bs[buf][1][w + 4 * u][l] = lo;
    }
    __syncthreads();
    // A of the next step before B of the step after it: loads complete in
    // order of issue, so the wait for the A operand leaves B in flight
    load_a(kk + 32, nh, nl);
    load_b(kk + 64, v);
    // keep the prefetches ahead of this step's products (the scheduler
    // would otherwise sink them below, leaving them no time in flight)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const u16x8 bh = Bs[buf][0][t][l], bl = Bs[buf][1][t][l];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) acc[rt][t] = mfma3(ah[rt], al[rt], bh, bl, acc[rt][t]);
    }
  };
  TB va[NS][8], vb[NS][8];
  u16x8 a0h[RT], a0l[RT], a1h[RT], a1l[RT];
  load_b(0, va);
  load_b(32, vb);
  load_a(0, a0h, a0l);
  const int nsteps = p.KP / 32;
  for (int kk = 0; kk + 64 <= 32 * nsteps; kk += 64) {
    step(kk, va, 0, a0h, a0l, a1h, a1l);
    step(kk + 32, vb, 1, a1h, a1l, a0h, a0l);
  }
  if (nsteps & 1) step(32 * (nsteps - 1), va, 0, a0h, a0l, a1h, a1l);
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = r0 + 16 * rt + 4 * (l >> 4) + i;
      if (row >= p.rows) continue;
      float *o = p.Out + static_cast<int64_t>(MAP ? p.map[row] : row) * p.ld;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int64_t s = s0 + 16 * t + (l & 15);
        if (s < p.count) o[s] = acc[rt][t][i];
      }
    }
}

template <int RT, int NT, bool BD, bool MAP>
__global__ __launch_bounds__(256) void k_lr_mfma(MfmaLrParams p) {
  lr_mfma_body<RT, NT, BD, MAP>(p, blockIdx.x, gridDim.x);
}

// Batched: slot = blockIdx.y; gridDim.x is a multiple of 8, so blockIdx.x
// mod 8 is still the XCD of the work-group.
template <int RT, int NT, bool BD, bool MAP>
__global__ __launch_bounds__(256) void k_lr_mfma_batch(const MfmaLrParams *ps) {
  const MfmaLrParams p = dev::load_uniform(ps + blockIdx.y);
  const unsigned total = static_cast<unsigned>((p.count + 16 * NT - 1) / (16 * NT)) *
                         static_cast<unsigned>((p.rows + 64 * RT - 1) / (64 * RT));
  if (blockIdx.x >= total) return;
  lr_mfma_body<RT, NT, BD, MAP>(p, blockIdx.x, total);
}

namespace {

template <int RT>
void launch_rt(hipStream_t s, const MfmaLrParams &p, dim3 grid, const LaunchEvents &ev) {
  if (p.Bd) {
    if (p.map) hipExtLaunchKernelGGL((k_lr_mfma<RT, kLrNT, true, true>), grid, dim3(256), 0, s, ev.start, ev.stop, 0, p);
    else hipExtLaunchKernelGGL((k_lr_mfma<RT, kLrNT, true, false>), grid, dim3(256), 0, s, ev.start, ev.stop, 0, p);
  } else {
    if (p.map) hipExtLaunchKernelGGL((k_lr_mfma<RT, kLrNT, false, true>), grid, dim3(256), 0, s, ev.start, ev.stop, 0, p);
    else hipExtLaunchKernelGGL((k_lr_mfma<RT, kLrNT, false, false>), grid, dim3(256), 0, s, ev.start, ev.stop, 0, p);
  }
}

template <int RT>
void launch_batch_rt(hipStream_t s, const MfmaLrParams *d, dim3 grid, bool bd, bool map) {
  if (bd) {
    if (map) hipLaunchKernelGGL((k_lr_mfma_batch<RT, kLrNT, true, true>), grid, dim3(256), 0, s, d);
    else hipLaunchKernelGGL((k_lr_mfma_batch<RT, kLrNT, true, false>), grid, dim3(256), 0, s, d);
  } else {
    if (map) hipLaunchKernelGGL((k_lr_mfma_batch<RT, kLrNT, false, true>), grid, dim3(256), 0, s, d);
    else hipLaunchKernelGGL((k_lr_mfma_batch<RT, kLrNT, false, false>), grid, dim3(256), 0, s, d);
  }
}

}  // namespace

void launch_lr_mfma(hipStream_t s, const MfmaLrParams &p, const LaunchEvents &ev) {
  const int rt = lr_mfma_rt(p.rows);
  const dim3 grid(lr_mfma_grid(p.count, p.rows).x);
  if (rt == 1) launch_rt<1>(s, p, grid, ev);
  else launch_rt<2>(s, p, grid, ev);
}

// Every descriptor of one batched launch must have lr_mfma_rt(rows) == rt
// and the same B type and map use; max_blocks bounds their block counts
// (lr_mfma_blocks).
void launch_lr_mfma_batch(hipStream_t s, const MfmaLrParams *d, int n, int rt, bool fp64_b, bool map,
                          int64_t max_blocks) {
  const Grid g = lr_mfma_batch_grid(n, max_blocks);
  const dim3 grid(g.x, g.y, g.z);
  if (rt == 1) launch_batch_rt<1>(s, d, grid, fp64_b, map);
  else launch_batch_rt<2>(s, d, grid, fp64_b, map);
}

}  // namespace tlrqmc

// HIP kernels of the TLR QMC sweep (gfx950), FP64 form.
//
// One lane = one sample.  Samples of a chunk are laid out contiguously in
// every per-sample buffer (Y, Delta, Z rows have leading dimension ld), so
// each wave reads and writes 64 consecutive doubles.  Factor entries are
// the same for every sample: their addresses depend only on loop counters
// and kernel arguments, so they are fetched once per wave with scalar loads.
//
// Per diagonal tile j (Section 3.4, TLR QMC for MVN: the dense MVN step on
// B_j after the limits of tile j were updated by the earlier tiles):
//   limit update: Delta_j = U_row(j) Z_row(j)  (FP64 matrix cores in
//                 kernels_lr64.hip; precision form in kernels_mfma.hip)
//   k_sweep     : the SOV recursion over the rows of B_j (Section 2.1, Eq. 2)
//   k_zproj_f64 : Z(:, j) = V_panel(j)^T Y_j    (rank-space image of y_j;
//                 precision form in kernels_mfma.hip)
// and k_reduce combines log P per shift (Section 2.1: mean over samples).
#include <hip/hip_ext.h>

#include <type_traits>

#include "device_math.hpp"
#include "internal.hpp"

namespace tlrqmc {

using namespace dev;

// w = ((W >> 12) + 1/2) 2^-52 for the Q0.64 point W = k A + D (mod 2^64):
// the 52 bits W >> 12 are the fraction of x = 1 + (W >> 12) 2^-52, and
// x - (1 - 2^-53) = ((W >> 12) + 1/2) 2^-52 exactly (the difference has at
// most 53 significant bits).
__device__ __forceinline__ double lattice_point(uint64_t k, uint64_t A, uint64_t D) {
  const uint64_t W = k * A + D;
  return __builtin_bit_cast(double, (W >> 12) | 0x3FF0000000000000ull) - (1.0 - 0x1p-53);
}

// ---------------------------------------------------------------- init ----
__device__ __forceinline__ void init_body(const InitParams &p, int64_t i) {
  if (i >= p.count) return;
  const int64_t g = p.g0 + i;
  p.logp[i] = 0.0;
  if (p.nu > 0.0) {
    const int64_t s = g / p.N;
    const uint64_t k = static_cast<uint64_t>(g - s * p.N) + 1;
    const double w0 = lattice_point(k, p.A[0], p.D[s * p.ldD]);
    p.R[i] = chi_inv(p.nu, w0) / sqrt(p.nu);
  }
}

__global__ __launch_bounds__(256) void k_init(InitParams p) {
  init_body(p, static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x);
}

// Batched launches (continuous batching of requests): one descriptor per
// slot, slot = blockIdx.y; the descriptor is read with scalar loads.
__global__ __launch_bounds__(256) void k_init_batch(const InitParams *ps) {
  const InitParams p = load_uniform(ps + blockIdx.y);
  init_body(p, static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x);
}

// --------------------------------------------------------------- sweep ----
// Blocked tile layout (row blocks of SB = kSweepBlock): for row block q the
// blocks (q, 0..q) are stored consecutively, SB*SB doubles each, starting
// at block index q(q+1)/2.  An off-diagonal block (q, p) is column-major:
// entry [u*SB + t] = B(SB q + t, SB p + u).  The diagonal block is stored by
// columns as well, entry [t*SB + i] = B(SB q + t + i, SB q + t) for i >= 1
// (zero past the block) and entry [t*SB] = 1 / B(SB q + t, SB q + t).
//
// Within a row block the recursion is right looking, in one of two forms
// that sum every row's terms in the same (increasing column) order, so
// they give identical results:
//  - the one-sided precision form unrolls the sixteen rows: acc[r] holds
//    the partial sum of row r of the block and, once y_t is known, column t
//    below the diagonal is added to rows t+1..15 only (no register moves;
//    a last, shorter block takes the rows it has by a wave-uniform branch);
//  - the other forms, whose FP64 special functions need more registers,
//    keep a sliding window: acc[i] holds the partial row sum of row t + i,
//    the whole column is added and the window moves down by one.
// Every index into acc is a compile-time constant, so acc stays in
// registers.
//
// The per-lane operands of a row (shift word, low-rank update) are loaded
// one row ahead and converted only when used, so that their memory latency
// overlaps the previous row's special functions.  The load is unconditional:
// a tile without a low-rank update reads a zero with zero strides.
//
// PREC selects the precision form: the low-rank update arrives in FP32, the
// one-sided step takes its special functions in FP32, and y is stored in FP32
// (its FP32 quantile is accurate to about 2e-7 already); the products with
// the diagonal tile stay FP64 arithmetic, on y widened back to FP64.
//
// Rows of earlier blocks enter through FP64 matrix cores: for row block q a
// wave forms C(64 samples x 16 rows) = sum_{p<q} Y_p(64 x 16) B(q,p)^T with
// v_mfma_f64_16x16x4_f64, four 16-sample tiles side by side.  The A operand
// is y of this wave's samples (lane l: sample 4*(l%16) + tile, block column
// 4*kstep + l/16, so that a lane's four tiles are four consecutive samples),
// the B operand is the factor block read once per k-step (lane l: entry
// [(4*kstep + l/16)*16 + l%16], contiguous).  The result leaves the matrix
// layout through a wave-private LDS tile (two halves of 32 samples) into the
// per-lane accumulator.  Every lane of a wave takes part; lanes past the
// chunk's end compute on clamped indices and store nothing outside their own
// Y column, which lies inside the leading dimension.
__device__ const double kNoDelta64 = 0.0;
__device__ const float kNoDelta32 = 0.0f;

template <class DT>
struct RowOperands {
  uint64_t d;
  DT dl;
};

template <class DT>
__device__ __forceinline__ RowOperands<DT> row_operands(const uint64_t *Ds, const DT *Dl, int64_t dls, int row) {
  return RowOperands<DT>{as_global(Ds)[row], as_global(Dl)[row * dls]};
}

typedef double f64x4 __attribute__((ext_vector_type(4)));

// Output layout of v_mfma_f64_16x16x4_f64: lane l holds column l % 16 and
// rows l / 16 + 4 r of the 16 x 16 tile, r = 0..3.
__device__ __forceinline__ int mfma64_row(int lane, int r) { return lane / 16 + 4 * r; }

constexpr int kTrLd = 18;  // LDS row stride of the transposition (doubles)

template <bool TWO_SIDED, bool SCALED, bool PREC>
__device__ __forceinline__ void sweep_body(const SweepParams &p, int64_t si, double *tr) {
  constexpr int SB = kSweepBlock;
  static_assert(SB == 16, "the matrix-core block products assume 16-row blocks");
  using DT = typename std::conditional<PREC, float, double>::type;  // low-rank update and y
  const int lane = static_cast<int>(threadIdx.x) & 63;
  const int64_t w0 = si - lane;
  if (w0 >= p.count) return;  // whole wave past the end
  // the same first sample, seen as wave-uniform (it keeps buffer resources
  // built from it in scalar registers)
  const int64_t w0u = static_cast<int64_t>(
      (static_cast<uint64_t>(static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(w0 >> 32)))) << 32) |
      static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(w0))));
  const bool live = si < p.count;
  const int64_t sl = live ? si : p.count - 1;
  const int64_t g = p.g0 + sl;
  const int64_t s = g / p.N;
  const uint64_t k = static_cast<uint64_t>(g - s * p.N) + 1;
  const uint64_t *Ds = p.D + s * p.ldD + p.c0;
  const auto Ag = as_const(p.A + p.c0);
  const auto bl = as_const(p.b);
  const auto al = as_const(p.a);
  const double R = SCALED ? p.R[sl] : 1.0;
  const int64_t ld = p.ld;
  DT *Y = static_cast<DT *>(p.Y) + si;
  const bool has_delta = p.Delta != nullptr;
  const DT *Dl = has_delta ? static_cast<const DT *>(p.Delta) + si
                           : (PREC ? reinterpret_cast<const DT *>(&kNoDelta32)
                                   : reinterpret_cast<const DT *>(&kNoDelta64));
  const int64_t dls = has_delta ? ld : 0;
  double lp = p.logp[sl];
  const int nb = (p.mj + SB - 1) / SB;
  auto blk = as_const(p.B);
  for (int q = 0; q < nb; ++q) {
    double acc[SB];
#pragma unroll
    for (int t = 0; t < SB; ++t) acc[t] = 0.0;
    if (q > 0) {
      f64x4 c[4];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) c[mt] = f64x4{0.0, 0.0, 0.0, 0.0};
      // Tile mt's A row i is sample 4 i + mt of the wave, so that lane l
      // reads samples 4 (l % 16) .. 4 (l % 16) + 3 of one y row in a single
      // 16-byte (FP64: two 16-byte) load.  The operands of block column
      // pb + 1 are loaded before the products of block column pb (the last
      // column loads itself again), so their latency overlaps the matrix
      // pipe.  The loads go through buffer resources over the block column
      // (16 y rows of the wave's samples; the q factor blocks of row block
      // q) with the k-step's offset in a scalar register; 16 ld elements
      // stay below 2 GiB (the drivers bound ld by 2^22).
      using V4 = DT __attribute__((ext_vector_type(4)));
      const uint32_t y_lane = static_cast<uint32_t>((static_cast<int64_t>(lane >> 4) * ld + 4 * (lane & 15)) * sizeof(DT));
      const uint32_t y_4rows = static_cast<uint32_t>(4 * ld * sizeof(DT));
      const int y_bytes = static_cast<int>(SB * ld * sizeof(DT));
      const double *Bq = p.B + static_cast<int64_t>(q) * (q + 1) / 2 * SB * SB;
      const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(Bq), 0, q * SB * SB * 8, kRawBufferWord3);
      auto load_col = [&](int pb, V4 (&ya)[4], double (&ba)[4]) {
        const __amdgpu_buffer_rsrc_t ry = __builtin_amdgcn_make_buffer_rsrc(
            static_cast<DT *>(p.Y) + w0u + static_cast<int64_t>(pb) * SB * ld, 0, y_bytes, kRawBufferWord3);
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const int so = static_cast<int>(ks * y_4rows);
          if constexpr (PREC) {
            ya[ks] = __builtin_bit_cast(V4, __builtin_amdgcn_raw_buffer_load_b128(ry, y_lane, so, 0));
          } else {
            typedef double f64x2 __attribute__((ext_vector_type(2)));
            const f64x2 lo = __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(ry, y_lane, so, 0));
            const f64x2 hi = __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(ry, y_lane + 16, so, 0));
            ya[ks] = V4{lo[0], lo[1], hi[0], hi[1]};
          }
          ba[ks] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rb, lane * 8, (pb * SB * SB + ks * 64) * 8, 0));
        }
      };
      auto products = [&](const V4 (&ya)[4], const double (&ba)[4]) {
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
#pragma unroll
          for (int mt = 0; mt < 4; ++mt)
            c[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(static_cast<double>(ya[ks][mt]), ba[ks], c[mt], 0, 0, 0);
      };
      V4 ya[4], yc[4];
      double ba[4], bc[4];
      load_col(0, ya, ba);
      for (int pb = 0; pb < q; ++pb) {
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          yc[ks] = ya[ks];
          bc[ks] = ba[ks];
        }
        load_col(min(pb + 1, q - 1), ya, ba);
        products(yc, bc);
      }
      blk += static_cast<int64_t>(q) * SB * SB;
      // matrix layout -> one lane per sample, 32 samples at a time (tile row
      // i of tile mt is sample 4 i + mt; rows r = 2h, 2h + 1 of every tile
      // hold samples 32 h .. 32 h + 31)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
          for (int r = 2 * h; r < 2 * h + 2; ++r)
            tr[(4 * mfma64_row(lane, r) + mt - 32 * h) * kTrLd + (lane & 15)] = c[mt][r];
        __builtin_amdgcn_wave_barrier();
        if ((lane >> 5) == h) {
#pragma unroll
          for (int t = 0; t < SB; ++t) acc[t] = tr[(lane & 31) * kTrLd + t];
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
    const int rows = min(SB, p.mj - q * SB);
    const int r0 = q * SB;
    RowOperands<DT> nxt = row_operands(Ds, Dl, dls, r0);
    // wave-uniform operands (limit, inverse diagonal, generator) of the next
    // row are fetched one row ahead, and the column below the diagonal
    // before the special functions that precede its use
    double bn = bl[r0], an = TWO_SIDED ? al[r0] : 0.0, dn = blk[0];
    uint64_t gn = Ag[r0];
    // Row t of the block: prefetch row t + 1's operands, then y_t from the
    // row's partial sum s (all its earlier terms).
    // The unrolled form (TRI) reads only the entries below the diagonal
    // (t is a compile-time constant there); the window reads the whole
    // column, whose entries past the block are zero.
    auto row_y = [&](int t, double s, double (&c)[SB], auto tri) -> double {
      const int row = r0 + t;
      const RowOperands<DT> cur = nxt;
      const double bc = bn, ac = an, dinv = dn;
      const uint64_t gc = gn;
      const auto col = blk + t * SB;
#pragma unroll
      for (int i = 1; i < SB; ++i)
        if (!decltype(tri)::value || t + i < SB) c[i] = col[i];
      if (t + 1 < rows) {
        nxt = row_operands(Ds, Dl, dls, row + 1);
        bn = bl[row + 1];
        if (TWO_SIDED) an = al[row + 1];
        dn = col[SB];
        gn = Ag[row + 1];
      }
      const double dl = static_cast<double>(cur.dl);
      const double bt = R * bc - dl;
      const double w = lattice_point(k, gc, cur.d);
      double y;
      if constexpr (TWO_SIDED) {
        const double at = R * ac - dl;
        lp += sov_step((at - s) * dinv, (bt - s) * dinv, w, y);
      } else {
        lp += PREC ? sov_step_upper_fp32((bt - s) * dinv, w, y) : sov_step_upper((bt - s) * dinv, w, y);
      }
      Y[row * ld] = static_cast<DT>(y);
      return y;
    };
    if constexpr (PREC && !TWO_SIDED) {
      // unrolled: column t below the diagonal goes to rows t+1..15 only
#pragma unroll
      for (int t = 0; t < SB; ++t) {
        if (t < rows) {
          double c[SB];
          const double y = row_y(t, acc[t], c, std::true_type{});
#pragma unroll
          for (int i = 1; t + i < SB; ++i) acc[t + i] = fma(c[i], y, acc[t + i]);
        }
      }
    } else {
      // sliding window (fewer registers for the FP64 special functions):
      // acc[i] holds the partial sum of row t + i; the window moves down by
      // one row per step (entries past the block are zero in the layout)
      for (int t = 0; t < rows; ++t) {
        double c[SB];
        const double y = row_y(t, acc[0], c, std::false_type{});
#pragma unroll
        for (int i = 1; i < SB; ++i) acc[i - 1] = fma(c[i], y, acc[i]);
        acc[SB - 1] = 0.0;
      }
    }
    blk += SB * SB;
  }
  if (live) p.logp[si] = lp;
}

template <bool TWO_SIDED, bool SCALED, bool PREC>
__global__ __launch_bounds__(256) void k_sweep(SweepParams p) {
  __shared__ double tr[4 * 32 * kTrLd];
  sweep_body<TWO_SIDED, SCALED, PREC>(p, static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x,
                                      tr + (threadIdx.x >> 6) * 32 * kTrLd);
}

template <bool TWO_SIDED, bool SCALED, bool PREC>
__global__ __launch_bounds__(256) void k_sweep_batch(const SweepParams *ps) {
  __shared__ double tr[4 * 32 * kTrLd];
  const SweepParams p = load_uniform(ps + blockIdx.y);
  sweep_body<TWO_SIDED, SCALED, PREC>(p, static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x,
                                      tr + (threadIdx.x >> 6) * 32 * kTrLd);
}

// ------------------------------------------------------- low rank, FP64 ----
// Z(map(c), s) = sum_t V_panel(t, c) Y(t, s) for 64 columns c per block row.
// V_panel is row-major with leading dimension lda (columns padded with zeros).
__device__ __forceinline__ void zproj_f64_body(const LrParams &p, int64_t si, int c0) {
  if (si >= p.count || c0 >= p.rows) return;
  double acc[kLrRows];
#pragma unroll
  for (int c = 0; c < kLrRows; ++c) acc[c] = 0.0;
  const double *Yv = p.In + si;
  const auto V = as_const(p.Mat + c0);
  const auto map = as_const(p.map);
#pragma unroll 2
  for (int t = 0; t < p.K; ++t) {
    const double y = Yv[static_cast<int64_t>(t) * p.ld];
    const auto Vt = V + static_cast<int64_t>(t) * p.lda;
#pragma unroll
    for (int c = 0; c < kLrRows; ++c) acc[c] = fma(Vt[c], y, acc[c]);
  }
  double *O = p.Out + si;
  const int nc = min(kLrRows, p.rows - c0);
#pragma unroll
  for (int c = 0; c < kLrRows; ++c)
    if (c < nc) O[static_cast<int64_t>(map[c0 + c]) * p.ld] = acc[c];
}

__global__ __launch_bounds__(256) void k_zproj_f64(LrParams p) {
  zproj_f64_body(p, static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x, blockIdx.y * kLrRows);
}

__global__ __launch_bounds__(256) void k_zproj_f64_batch(const LrParams *ps) {
  const LrParams p = load_uniform(ps + blockIdx.z);
  zproj_f64_body(p, static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x, blockIdx.y * kLrRows);
}

// -------------------------------------------------------------- reduce ----
// One block per shift: max of log P, then sum of exp(log P - max) and the
// count of empty samples.  Each lane strides over the samples in a fixed
// order; a wave combines its lanes by a butterfly of lane exchanges (lane i
// and lane i ^ d add the same two values, so every lane ends with the same
// sum), and the four waves' results are combined in a fixed order, so the
// result does not depend on scheduling.
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v = fmax(v, __shfl_xor(v, d, 64));
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ void reduce_body(const ReduceParams &p, int s, double *sh) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const double *lp = p.logp + static_cast<int64_t>(s) * p.N;
  double mx = -INFINITY;
  for (int64_t i = t; i < p.N; i += 256) mx = fmax(mx, lp[i]);
  mx = wave_max(mx);
  if (lane == 0) sh[w] = mx;
  __syncthreads();
  mx = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
  double sum = 0.0, dead = 0.0;
  if (mx > -INFINITY) {
    for (int64_t i = t; i < p.N; i += 256) {
      const double v = lp[i];
      sum += exp(v - mx);
      dead += (v == -INFINITY) ? 1.0 : 0.0;
    }
  } else {
    for (int64_t i = t; i < p.N; i += 256) dead += 1.0;
  }
  sum = wave_sum(sum);
  dead = wave_sum(dead);
  if (lane == 0) {
    sh[4 + w] = sum;
    sh[8 + w] = dead;
  }
  __syncthreads();
  if (t == 0) {
    p.part[3 * s + 0] = mx;
    p.part[3 * s + 1] = (sh[4] + sh[5]) + (sh[6] + sh[7]);
    p.part[3 * s + 2] = (sh[8] + sh[9]) + (sh[10] + sh[11]);
  }
}

__global__ __launch_bounds__(256) void k_reduce(ReduceParams p) {
  __shared__ double sh[12];
  reduce_body(p, blockIdx.x, sh);
}

// One block per (shift, request); blocks past a request's shift count
// leave at once (the whole block takes the same branch).
__global__ __launch_bounds__(256) void k_reduce_batch(const ReduceParams *ps) {
  __shared__ double sh[12];
  const ReduceParams p = load_uniform(ps + blockIdx.y);
  if (static_cast<int>(blockIdx.x) >= p.M) return;
  reduce_body(p, blockIdx.x, sh);
}

// ------------------------------------------------------------ launchers ----
static inline dim3 dim3_of(const Grid &g) { return dim3(g.x, g.y, g.z); }

void launch_init(hipStream_t s, const InitParams &p, const LaunchEvents &ev) {
  hipExtLaunchKernelGGL(k_init, dim3_of(init_grid(p.count)), dim3(256), 0, s, ev.start, ev.stop, 0, p);
}

template <bool TWO_SIDED, bool SCALED>
static void sweep_form(hipStream_t s, const SweepParams &p, dim3 grid, bool prec, const LaunchEvents &ev) {
  if (prec) hipExtLaunchKernelGGL((k_sweep<TWO_SIDED, SCALED, true>), grid, dim3(256), 0, s, ev.start, ev.stop, 0, p);
  else hipExtLaunchKernelGGL((k_sweep<TWO_SIDED, SCALED, false>), grid, dim3(256), 0, s, ev.start, ev.stop, 0, p);
}

void launch_sweep(hipStream_t s, const SweepParams &p, bool two_sided, bool scaled, bool prec,
                  const LaunchEvents &ev) {
  const dim3 grid = dim3_of(sweep_grid(p.count));
  if (two_sided) {
    if (scaled) sweep_form<true, true>(s, p, grid, prec, ev);
    else sweep_form<true, false>(s, p, grid, prec, ev);
  } else {
    if (scaled) sweep_form<false, true>(s, p, grid, prec, ev);
    else sweep_form<false, false>(s, p, grid, prec, ev);
  }
}

void launch_zproj_f64(hipStream_t s, const LrParams &p, const LaunchEvents &ev) {
  hipExtLaunchKernelGGL(k_zproj_f64, dim3_of(zproj_f64_grid(p.count, p.rows)), dim3(256), 0, s, ev.start, ev.stop, 0, p);
}

void launch_reduce(hipStream_t s, const ReduceParams &p, int n_shifts, const LaunchEvents &ev) {
  hipExtLaunchKernelGGL(k_reduce, dim3_of(reduce_grid(n_shifts)), dim3(256), 0, s, ev.start, ev.stop, 0, p);
}

void launch_init_batch(hipStream_t s, const InitParams *d, int n, int64_t max_count) {
  hipLaunchKernelGGL(k_init_batch, dim3_of(init_batch_grid(n, max_count)), dim3(256), 0, s, d);
}

template <bool TWO_SIDED, bool SCALED>
static void sweep_batch_form(hipStream_t s, const SweepParams *d, dim3 grid, bool prec) {
  if (prec) hipLaunchKernelGGL((k_sweep_batch<TWO_SIDED, SCALED, true>), grid, dim3(256), 0, s, d);
  else hipLaunchKernelGGL((k_sweep_batch<TWO_SIDED, SCALED, false>), grid, dim3(256), 0, s, d);
}

void launch_sweep_batch(hipStream_t s, const SweepParams *d, int n, int64_t max_count, bool two_sided, bool scaled,
                        bool prec) {
  const dim3 grid = dim3_of(sweep_batch_grid(n, max_count));
  if (two_sided) {
    if (scaled) sweep_batch_form<true, true>(s, d, grid, prec);
    else sweep_batch_form<true, false>(s, d, grid, prec);
  } else {
    if (scaled) sweep_batch_form<false, true>(s, d, grid, prec);
    else sweep_batch_form<false, false>(s, d, grid, prec);
  }
}

void launch_zproj_f64_batch(hipStream_t s, const LrParams *d, int n, int64_t max_count, int max_rows) {
  hipLaunchKernelGGL(k_zproj_f64_batch, dim3_of(zproj_f64_batch_grid(n, max_count, max_rows)), dim3(256), 0, s, d);
}

void launch_reduce_batch(hipStream_t s, const ReduceParams *d, int n, int max_shifts) {
  hipLaunchKernelGGL(k_reduce_batch, dim3_of(reduce_batch_grid(n, max_shifts)), dim3(256), 0, s, d);
}

}  // namespace tlrqmc

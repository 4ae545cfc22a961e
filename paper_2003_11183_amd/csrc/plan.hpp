// Host-side plan of the estimator: the device layout of a factor, the
// per-chunk buffers, the descriptors of every launch of a tile step and the
// launch grids.  Plain C++ without the HIP runtime: the estimator driver,
// the request server and the address replay of the test suite all build
// their launches from these functions.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "tlrqmc.h"

namespace tlrqmc {

// Row-block height of the diagonal-tile sweep.
constexpr int kSweepBlock = 16;
// Rows (delta) / columns (projection) produced per FP64 low-rank pass.
constexpr int kLrRows = 64;
// Rows and samples of one work-group of the FP64 matrix-core limit update.
constexpr int kLr64Tile = 128;
// Sample tiles of 16 per work-group of the BF16 low-rank kernel (128 samples).
constexpr int kLrNT = 8;

inline int64_t round_up(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

// ---- kernel descriptors (passed by value, or as device arrays in batches) ----
struct InitParams {
  int64_t g0, count, N;
  const uint64_t *A, *D;   // generators, shift table (ldD per shift)
  int64_t ldD;
  double nu;               // 0 = normal
  double *logp;            // per chunk sample
  double *R;               // per chunk sample (nu > 0)
};

struct SweepParams {
  int64_t g0, count, N, ld, ldD;
  int mj, c0;              // rows of the tile, lattice coordinate of row 0
  const double *B;         // blocked tile
  const double *a, *b;     // limits of the tile rows (a unused when one-sided)
  const void *Delta;       // m x ld low-rank update (FP32 in the precision form, FP64 otherwise), or null
  const double *R;         // per chunk sample, or null
  const uint64_t *A, *D;
  double *logp;            // per chunk sample
  void *Y;                 // tile rows x ld: FP32 in the precision form, FP64 otherwise
};

struct LrParams {
  int64_t count, ld;
  int rows, K;             // delta: rows = m_i, K = krow; zproj: rows = K_col, K = m_j
  int lda;                 // padded leading dimension of the tile operand
  const double *Mat;       // U_row (col-major, lda rows) or V_panel (row-major, lda cols)
  const double *In;        // Z rows (delta) or Y (zproj), ld-strided
  double *Out;             // Delta (delta) or Z (zproj)
  const int32_t *map;      // zproj: output row map
};

struct ReduceParams {
  int64_t N;
  int M;                   // shifts (blocks), read by the batched launch
  const double *logp;
  double *part;            // per shift: max, sum exp(lp - max), dead count
};

// C (rows x count) = A (rows x K) B (K x count) on BF16 matrix cores.  A is
// pre-split into BF16 hi/lo, row-major with leading dimension KP (a
// multiple of 32), rows padded to lr_mfma_rows(rows); B is FP32 or FP64
// with leading dimension ld.  Output row c goes to row map[c] when a map
// is given.
struct MfmaLrParams {
  int64_t count, ld;
  int rows, K, KP;
  const unsigned short *Ahi, *Alo;
  const float *Bf;         // B in FP32, or null
  const double *Bd;        // B in FP64, or null
  const int32_t *map;      // output row map, or null
  float *Out;
};

// ---- launch grids (blocks of 256 threads) ----
struct Grid {
  unsigned x = 1, y = 1, z = 1;
};

inline unsigned grid_of(int64_t count) { return static_cast<unsigned>((count + 255) / 256); }

// Row tiles of 16 per wave of the BF16 low-rank kernel: one for operands
// of at most 64 rows, else two (measured at n = 16,384 against four, with
// 64-, 128- and 256-sample blocks: 128 samples and two row tiles were
// fastest for both products).
inline int lr_mfma_rt(int rows) { return rows <= 64 ? 1 : 2; }
// Rows of the kernel's A operand (rows padded to its row block).
inline int64_t lr_mfma_rows(int rows) { return round_up(rows > 0 ? rows : 1, 64 * lr_mfma_rt(rows)); }
// Work-groups of one launch over count samples and rows rows.
inline int64_t lr_mfma_blocks(int64_t count, int rows) {
  const int rt = lr_mfma_rt(rows);
  return (count + 16 * kLrNT - 1) / (16 * kLrNT) * ((rows + 64 * rt - 1) / (64 * rt));
}

inline Grid init_grid(int64_t count) { return {grid_of(count), 1, 1}; }
inline Grid sweep_grid(int64_t count) { return {grid_of(count), 1, 1}; }
inline Grid zproj_f64_grid(int64_t count, int rows) {
  return {grid_of(count), static_cast<unsigned>((rows + kLrRows - 1) / kLrRows), 1};
}
inline Grid lr64_grid(int64_t count, int rows, int n) {
  return {static_cast<unsigned>((count + kLr64Tile - 1) / kLr64Tile),
          static_cast<unsigned>((rows + kLr64Tile - 1) / kLr64Tile), static_cast<unsigned>(n)};
}
inline Grid lr_mfma_grid(int64_t count, int rows) { return {static_cast<unsigned>(lr_mfma_blocks(count, rows)), 1, 1}; }
inline Grid reduce_grid(int n_shifts) { return {static_cast<unsigned>(n_shifts), 1, 1}; }
// Batched launches: one descriptor per slot; the grid covers the largest.
inline Grid init_batch_grid(int n, int64_t max_count) { return {grid_of(max_count), static_cast<unsigned>(n), 1}; }
inline Grid sweep_batch_grid(int n, int64_t max_count) { return {grid_of(max_count), static_cast<unsigned>(n), 1}; }
inline Grid zproj_f64_batch_grid(int n, int64_t max_count, int max_rows) {
  Grid g = zproj_f64_grid(max_count, max_rows);
  g.z = static_cast<unsigned>(n);
  return g;
}
inline Grid lr64_batch_grid(int n, int64_t max_count, int max_rows) { return lr64_grid(max_count, max_rows, n); }
inline Grid reduce_batch_grid(int n, int max_shifts) {
  return {static_cast<unsigned>(max_shifts), static_cast<unsigned>(n), 1};
}
// gridDim.x a multiple of 8, so that blockIdx.x mod 8 is the XCD of a work-group
inline Grid lr_mfma_batch_grid(int n, int64_t max_blocks) {
  return {static_cast<unsigned>(round_up(max_blocks, 8)), static_cast<unsigned>(n), 1};
}

}  // namespace tlrqmc

// Device-resident TLR factor.  Host vectors keep the exchange layout for
// export and the sizes the launches need.
struct tlrqmc_factor {
  tlrqmc_ctx *ctx = nullptr;
  int64_t n = 0;
  int m = 0, r = 0;
  std::vector<int32_t> perm;
  std::vector<int> tm;          // rows of tile i
  std::vector<int64_t> toff;    // first variable of tile i
  std::vector<int32_t> rank;    // r x r, rank[i*r+j] for i > j
  std::vector<int64_t> krow;    // sum_j<i k_ij: width of U_row(i)
  std::vector<int64_t> kcol;    // sum_i>j k_ij: width of V_panel(j)
  std::vector<int64_t> zoff;    // first Z row of tile i (prefix of krow)
  int64_t k_tot = 0;
  int k_max = 0;
  int cap_hits = 0;
  // Host exchange copies.
  std::vector<double> h_diag, h_U, h_V;
  // Device layouts.
  double *d_diag = nullptr;     // blocked diagonal tiles (see kernels)
  std::vector<int64_t> diag_off;
  double *d_urow = nullptr;     // U_row(i): column-major, rows padded to kLrRows
  std::vector<int64_t> urow_off;
  std::vector<int> urow_ld;
  double *d_vpan = nullptr;     // V_panel(j): row-major, columns padded to kLrRows
  std::vector<int64_t> vpan_off;
  std::vector<int> vpan_ld;
  int32_t *d_zmap = nullptr;    // V_panel(j) column -> Z row
  std::vector<int64_t> zmap_off;
  uint64_t *d_gen = nullptr;    // lattice generators A_0..A_n
  // Precision form: BF16 hi/lo splits of U_row (row-major, k padded to 32,
  // rows padded to the MFMA block) and of V_panel^T (row-major, t padded to
  // 32), and a Z layout whose row blocks are padded to 32.
  unsigned short *d_ubf = nullptr;
  std::vector<int64_t> ubf_off;  // hi at off, lo at off + ubf_size[i]
  std::vector<int64_t> ubf_size;
  std::vector<int> kp_row;       // round_up(krow, 32)
  unsigned short *d_vbf = nullptr;
  std::vector<int64_t> vbf_off;
  std::vector<int64_t> vbf_size;
  std::vector<int> vbf_mp;       // round_up(m_j, 32)
  int32_t *d_zmapp = nullptr;    // V_panel(j) column -> padded Z row
  std::vector<int64_t> zoffp;    // first padded Z row of tile i
  int64_t zp_tot = 0;
  int64_t device_bytes = 0;
  double setup_seconds[4] = {0, 0, 0, 0};  // tlr_factor phases
  uint64_t checksum = 0;                   // FNV-1a of perm, diag, ranks, U, V
  int64_t host_tiles = 0;                  // off-diagonal tiles compressed on the host
};

namespace tlrqmc {

// ---- factor layout ----
// Tile geometry and ranks of a factor (n, m, r, tm, toff, rank, krow, kcol,
// zoff, k_tot, k_max) from validated ranks (r x r, entries i > j).
void factor_geometry(tlrqmc_factor *f, int64_t n, int m, const int32_t *ranks);
// Offsets of every device array from the geometry (diag_off .. zp_tot).
void factor_layout(tlrqmc_factor *f);
// Bytes of the eight device arrays: diagonal tiles, U_row, V_panel, zmap,
// generators, BF16 U, BF16 V, padded zmap.
void factor_device_sizes(const tlrqmc_factor *f, size_t sizes[8]);
// Z row (z) and padded Z row (zp) of every column of V_panel(i).
void factor_zmaps(const tlrqmc_factor *f, int i, int32_t *z, int32_t *zp);

// ---- chunk buffers ----
// Per-chunk device buffers: Y (tile rows x ld), the low-rank update of a
// tile, the rank-space images Z, the chi radii.  FP32 in the precision
// form for Y, the update and Z.
struct ChunkBuffers {
  void *Y = nullptr;
  double *Dl = nullptr, *Z = nullptr, *R = nullptr;
  float *DlF = nullptr, *ZF = nullptr;
};
// Bytes of Y, the update, Z and R for a chunk of leading dimension ld (0
// where the chunk has no such buffer), in the order the drivers take them.
void chunk_buffer_bytes(const tlrqmc_factor *f, bool prec, bool scaled, int64_t ld, int64_t bytes[4]);
// Device bytes per sample of a chunk, an upper bound of the above over ld
// (the chi radii counted whether or not they are needed).
int64_t chunk_bytes_per_sample(const tlrqmc_factor *f, bool prec);

// ---- chunking of one estimator call ----
// Samples per call from which the chunks run on two worker streams, the
// device memory the chunk buffers may take, and the largest chunk (the
// low-rank kernels address 32 rows of a chunk buffer with 32-bit byte
// offsets).
constexpr int64_t kMultiStreamSamples = 131072;
constexpr int kWorkerStreams = 2;
constexpr int64_t kScratchBudget = int64_t{64} << 30;
constexpr int64_t kMaxChunk = int64_t{1} << 22;
// Bytes of the per-call arrays (limits, shift table, log P per sample, the
// per-shift partial sums), each rounded up to 256, taken before the chunk
// buffers.
int64_t estimator_call_bytes(int64_t n, int M, int64_t count, bool two_sided, bool reduce);
struct ChunkPlan {
  int nstream;
  int64_t chunk;  // samples per chunk = leading dimension (a multiple of 256); 0: does not fit
};
// Chunks of a call over count samples: requested samples per chunk (0 =
// choose), fixed_left the bytes of a fixed region that must hold every
// buffer (negative: the allocator, with two worker streams for large
// calls).
ChunkPlan plan_chunks(const tlrqmc_factor *f, bool prec, int64_t count, int64_t requested, int64_t fixed_left,
                      int64_t call_bytes);

// ---- slots of a served request ----
// Samples per slot at most, and the device bytes one slot's buffers may
// take; a request's slots all have the same size.
constexpr int64_t kSlotSamples = 32768;
constexpr int64_t kSlotBytes = int64_t{2} << 30;
struct SlotPlan {
  int64_t chunk;       // samples per slot = leading dimension (a multiple of 256)
  int nslots;
  int64_t slot_bytes;  // the slot's buffers, each rounded up to 256
};
SlotPlan plan_slots(const tlrqmc_factor *f, bool prec, bool scaled, int64_t count);

// ---- one tile step of one chunk ----
// Samples g0 .. g0 + count - 1 (of the flattened shift-major index) in
// chunk buffers of leading dimension ld; a and b are the limits in
// integration order (a null when one-sided), D the shift table, logp the
// chunk's first sample.
struct ChunkRun {
  int64_t g0, count, N, ld;
  bool prec;
  ChunkBuffers buf;
  const double *a, *b;
  const uint64_t *D;
  double *logp;
};
struct TileLaunch {
  bool delta = false, zproj = false;
  MfmaLrParams delta_mfma{}, zproj_mfma{};  // precision form
  LrParams delta_f64{}, zproj_f64{};        // FP64 form
  SweepParams sweep{};
};
// The launches of tile j: limit update (j > 0 with a nonzero row rank),
// sweep, projection (j < r - 1 with a nonzero column rank).
TileLaunch tile_launch(const tlrqmc_factor *f, int j, const ChunkRun &c);
InitParams init_launch(const tlrqmc_factor *f, const ChunkRun &c, double nu);

}  // namespace tlrqmc

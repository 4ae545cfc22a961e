// Setup-side declarations: launchers of the setup kernels (dense Cholesky,
// tile compression), the sizes of their buffers, and factor assembly from
// vectors the factor takes over.  Kept apart from internal.hpp, which the
// estimator kernels include.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

struct tlrqmc_ctx;
struct tlrqmc_factor;

namespace tlrqmc {

// ---- dense Cholesky on the device (kernels_chol.hip) ----
// L L^T = A in place (lower, column-major, leading dimension lda); *info
// must be zero on entry and receives the 1-based row of the first
// non-positive pivot.  scratch holds kCholScratch doubles.
constexpr int kCholBlock = 64;
constexpr int kCholPanel = 256;  // columns per trailing update (a multiple of kCholBlock)
constexpr int64_t kCholScratch = kCholBlock * kCholBlock + kCholBlock;
void launch_cholesky(hipStream_t s, double *A, int64_t lda, int64_t n, int32_t *info, double *scratch);

// Device compression of the off-diagonal tiles of a dense factor
// (kernels_compress.hip).  Tiles are numbered in row order, t = i (i - 1) / 2
// + j for j < i; one launch handles tiles t0 .. t0 + count - 1.  Per tile, W
// holds m * m doubles and Vs compress_vslot(m); out receives the batch's U
// blocks, then its V blocks, packed in tile order (at most 2 compress_vslot(m)
// doubles per tile); info holds four ints per tile: QR steps, rank, flags
// (1 = more than kCmpKq QR steps needed, compress on the host; 2 = rank
// capped).  Tiles wider than kCmpMaxTile are compressed on the host.
constexpr int kCmpKq = 96;
constexpr int kCmpMaxTile = 512;
void launch_compress(hipStream_t s, const double *L, int64_t lda, int64_t n, int m, int64_t t0, int count,
                     double tol, int cap, double *W, double *Vs, double *out, int32_t *info);
void compress_tile_at(int64_t t, int64_t n, int m, int64_t &row0, int64_t &col0, int &mi, int &mj);
// Doubles of a tile's V buffer (a rank never exceeds min(m, kCmpKq)), tiles
// per device compression batch, and the device bytes of a batch's buffers
// (W, V, the packed output of twice the V size, info).
inline int64_t compress_vslot(int m) { return static_cast<int64_t>(m) * std::min(m, kCmpKq); }
inline int64_t compress_slot_bytes(int m) { return 8 * (static_cast<int64_t>(m) * m + 3 * compress_vslot(m)) + 16; }
inline int64_t compress_batch_tiles(int64_t n, int m) {
  const int64_t r = (n + m - 1) / m, tiles = r * (r - 1) / 2;
  return std::min(tiles, std::max<int64_t>(256, (int64_t{1} << 30) / compress_slot_bytes(m)));
}
inline int64_t compress_scratch_bytes(int64_t n, int m) {
  if (m > kCmpMaxTile) return 0;
  return compress_batch_tiles(n, m) * compress_slot_bytes(m) + 4 * 256;
}

// factor_build (factor.cpp) taking diag, U and V over instead of copying
// them when their sizes are those the ranks imply (the vectors may then be
// left empty); arguments otherwise as for factor_build.
int factor_build_take(tlrqmc_ctx *ctx, int64_t n, int m, const int32_t *perm, std::vector<double> &diag,
                      const int32_t *ranks, std::vector<double> &U, std::vector<double> &V, int cap_hits,
                      tlrqmc_factor **out);

}  // namespace tlrqmc

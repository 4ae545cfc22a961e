// Factor construction: exchange layout on the host -> device layouts.
//
// The TLR factor of Section 3.4 is r diagonal tiles B_i and off-diagonal
// tiles L_ij = U_ij V_ij^T (i > j).  The estimator walks the tiles left
// looking: Delta_i = sum_j<i U_ij (V_ij^T y_j) = U_row(i) Z_row(i), where
// U_row(i) = [U_i0 ... U_i,i-1] and Z_row(i) stacks the rank-space images
// V_ij^T y_j.  Those images are produced right after tile j by one product
// with V_panel(j) = [V_j+1,j ... V_r-1,j]; zmap sends each of its columns
// to the row of Z_row(i) it belongs to.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>

#include "internal.hpp"
#include "setup_kernels.hpp"

namespace tlrqmc {

namespace {

// x = hi + lo with hi = bf16(float(x)), lo = bf16(float(x - hi)), both
// rounded to nearest even.
void split_bf16(double x, unsigned short &hi, unsigned short &lo) {
  auto bits = [](float v) {
    uint32_t u;
    std::memcpy(&u, &v, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<unsigned short>(u >> 16);
  };
  hi = bits(static_cast<float>(x));
  const uint32_t hb = static_cast<uint32_t>(hi) << 16;
  float hf;
  std::memcpy(&hf, &hb, 4);
  lo = bits(static_cast<float>(x - static_cast<double>(hf)));
}

}  // namespace

namespace {

// own_*: when given with the sizes the ranks imply, the host exchange copies
// are taken from these vectors (left empty) instead of copied.
int build_impl(tlrqmc_ctx *ctx, int64_t n, int m, const int32_t *perm, const double *diag, const int32_t *ranks,
               const double *U, const double *V, int cap_hits, std::vector<double> *own_diag,
               std::vector<double> *own_U, std::vector<double> *own_V, tlrqmc_factor **out) {
  if (!ctx || !out) return fail(TLRQMC_EINVAL, "null context or output pointer");
  *out = nullptr;
  if (n < 1 || m < 1) return fail(TLRQMC_EINVAL, "n and m must be positive (n=%lld, m=%d)",
                                  static_cast<long long>(n), m);
  if (n > (int64_t{1} << 30)) return fail(TLRQMC_EINVAL, "n too large");
  if (!diag || !ranks) return fail(TLRQMC_EINVAL, "diag and ranks are required");
  const int r = static_cast<int>((n + m - 1) / m);
  auto f = new tlrqmc_factor();
  std::unique_ptr<tlrqmc_factor, void (*)(tlrqmc_factor *)> guard(f, tlrqmc_factor_free);
  f->ctx = ctx;
  f->cap_hits = cap_hits;
  f->perm.resize(n);
  if (perm) {
    std::vector<uint8_t> seen(n, 0);
    for (int64_t i = 0; i < n; ++i) {
      const int32_t v = perm[i];
      if (v < 0 || v >= n || seen[v]) return fail(TLRQMC_EINVAL, "perm is not a permutation (entry %lld)", static_cast<long long>(i));
      seen[v] = 1;
      f->perm[i] = v;
    }
  } else {
    std::iota(f->perm.begin(), f->perm.end(), 0);
  }
  // ranks, then the tile geometry and the derived widths
  auto rows_of = [&](int i) { return static_cast<int>(std::min<int64_t>(m, n - static_cast<int64_t>(i) * m)); };
  int64_t uv_doubles_u = 0, uv_doubles_v = 0;
  for (int i = 1; i < r; ++i)
    for (int j = 0; j < i; ++j) {
      const int k = ranks[static_cast<size_t>(i) * r + j];
      if (k < 0 || k > std::min(rows_of(i), rows_of(j)))
        return fail(TLRQMC_EINVAL, "rank of tile (%d,%d) out of range: %d", i, j, k);
      if (k > 0 && (!U || !V)) return fail(TLRQMC_EINVAL, "U and V are required for nonzero ranks");
      uv_doubles_u += static_cast<int64_t>(rows_of(i)) * k;
      uv_doubles_v += static_cast<int64_t>(rows_of(j)) * k;
    }
  factor_geometry(f, n, m, ranks);
  if (f->k_tot > (int64_t{1} << 31) - 1) return fail(TLRQMC_EINVAL, "total rank too large");
  // host exchange copies (validated)
  int64_t diag_doubles = 0;
  for (int i = 0; i < r; ++i) diag_doubles += static_cast<int64_t>(f->tm[i]) * f->tm[i];
  if (own_diag && static_cast<int64_t>(own_diag->size()) == diag_doubles && own_U &&
      static_cast<int64_t>(own_U->size()) == uv_doubles_u && own_V &&
      static_cast<int64_t>(own_V->size()) == uv_doubles_v) {
    f->h_diag.swap(*own_diag);
    f->h_U.swap(*own_U);
    f->h_V.swap(*own_V);
  } else {
    f->h_diag.assign(diag, diag + diag_doubles);
    if (uv_doubles_u) {
      f->h_U.assign(U, U + uv_doubles_u);
      f->h_V.assign(V, V + uv_doubles_v);
    }
  }
  {
    std::vector<int64_t> o(r + 1, 0);
    for (int i = 0; i < r; ++i) o[i + 1] = o[i] + static_cast<int64_t>(f->tm[i]) * f->tm[i];
    // per tile: 0 = valid, 1 = non-finite entry, 2 + t = non-positive pivot t
    std::vector<int64_t> verdict(r, 0);
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < r; ++i) {
      const int mi = f->tm[i];
      const double *D = f->h_diag.data() + o[i];
      for (int t = 0; t < mi && !verdict[i]; ++t) {
        for (int u = 0; u <= t; ++u)
          if (!std::isfinite(D[static_cast<int64_t>(t) * mi + u])) verdict[i] = 1;
        if (!verdict[i] && !(D[static_cast<int64_t>(t) * mi + t] > 0.0)) verdict[i] = 2 + t;
      }
    }
    for (int i = 0; i < r; ++i) {
      if (verdict[i] == 1) return fail(TLRQMC_EINVAL, "non-finite diagonal-tile entry in tile %d", i);
      if (verdict[i] >= 2)
        return fail(TLRQMC_EINVAL, "diagonal entry %lld is not positive",
                    static_cast<long long>(f->toff[i] + verdict[i] - 2));
    }
    int bad = 0;
    const int64_t nu = static_cast<int64_t>(f->h_U.size()), nv = static_cast<int64_t>(f->h_V.size());
#pragma omp parallel for reduction(| : bad)
    for (int64_t q = 0; q < nu; ++q) bad |= std::isfinite(f->h_U[q]) ? 0 : 1;
    if (bad) return fail(TLRQMC_EINVAL, "non-finite entry in U");
#pragma omp parallel for reduction(| : bad)
    for (int64_t q = 0; q < nv; ++q) bad |= std::isfinite(f->h_V[q]) ? 0 : 2;
    if (bad) return fail(TLRQMC_EINVAL, "non-finite entry in V");
  }
  // Offsets first, then every tile's layout in parallel (tiles are
  // independent).
  constexpr int SB = kSweepBlock;
  std::vector<int64_t> dsrc(r + 1, 0);
  for (int i = 0; i < r; ++i) dsrc[i + 1] = dsrc[i] + static_cast<int64_t>(f->tm[i]) * f->tm[i];
  std::vector<int64_t> u_src(static_cast<size_t>(r) * r, 0), v_src(static_cast<size_t>(r) * r, 0);
  {
    int64_t ou = 0, ov = 0;
    for (int i = 1; i < r; ++i)
      for (int j = 0; j < i; ++j) {
        const int k = f->rank[static_cast<size_t>(i) * r + j];
        u_src[static_cast<size_t>(i) * r + j] = ou;
        v_src[static_cast<size_t>(i) * r + j] = ov;
        ou += static_cast<int64_t>(f->tm[i]) * k;
        ov += static_cast<int64_t>(f->tm[j]) * k;
      }
  }
  factor_layout(f);
  // Every device array is laid out directly in one pinned staging buffer
  // (already mapped, so no page faults), cleared in parallel, filled tile by
  // tile, then uploaded.
  const std::vector<uint64_t> gen = richtmyer_generators(n + 1);
  size_t sizes[8];
  factor_device_sizes(f, sizes);
  size_t offs[9] = {0};
  for (int k = 0; k < 8; ++k) offs[k + 1] = offs[k] + static_cast<size_t>(round_up(static_cast<int64_t>(sizes[k]), 256));
  char *stage = reinterpret_cast<char *>(ctx->pinned(2, offs[8]));
  if (!stage) return fail(TLRQMC_ENOMEM, "pinned host staging allocation failed");
  {
    const int64_t words = static_cast<int64_t>(offs[8] / 8);
    uint64_t *w = reinterpret_cast<uint64_t *>(stage);
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < words; ++q) w[q] = 0;
  }
  double *hb = reinterpret_cast<double *>(stage + offs[0]);
  double *hu = reinterpret_cast<double *>(stage + offs[1]);
  double *hv = reinterpret_cast<double *>(stage + offs[2]);
  int32_t *hz = reinterpret_cast<int32_t *>(stage + offs[3]);
  std::memcpy(stage + offs[4], gen.data(), sizes[4]);
  unsigned short *hub = reinterpret_cast<unsigned short *>(stage + offs[5]);
  unsigned short *hvb = reinterpret_cast<unsigned short *>(stage + offs[6]);
  int32_t *hzp = reinterpret_cast<int32_t *>(stage + offs[7]);
#pragma omp parallel for schedule(dynamic, 1)
  for (int i = 0; i < r; ++i) {
    // blocked diagonal tile (row blocks of SB, see the sweep kernel)
    const int mi = f->tm[i];
    const int nb = (mi + SB - 1) / SB;
    double *T = hb + f->diag_off[i];
    const double *src = f->h_diag.data() + dsrc[i];
    auto Bat = [&](int t, int u) { return src[static_cast<int64_t>(t) * mi + u]; };
    for (int q = 0; q < nb; ++q)
      for (int pb = 0; pb <= q; ++pb) {
        double *blk = T + (static_cast<int64_t>(q) * (q + 1) / 2 + pb) * SB * SB;
        if (pb < q) {
          for (int u = 0; u < SB; ++u)
            for (int t = 0; t < SB; ++t) {
              const int row = SB * q + t, c = SB * pb + u;
              blk[u * SB + t] = row < mi ? Bat(row, c) : 0.0;
            }
        } else {
          for (int t = 0; t < SB; ++t) {
            const int row = SB * q + t;
            if (row >= mi) continue;
            blk[t * SB] = 1.0 / Bat(row, row);
            for (int ii = 1; t + ii < SB; ++ii)
              if (row + ii < mi) blk[t * SB + ii] = Bat(row + ii, row);
          }
        }
      }
    // U_row(i): column-major, rows padded to kLrRows; its BF16 split
    // row-major with k padded to 32
    const int lda = f->urow_ld[i];
    double *du = hu + f->urow_off[i];
    const int64_t kp = f->kp_row[i];
    unsigned short *hi = hub + f->ubf_off[i], *lo = hi + f->ubf_size[i];
    int64_t col = 0;
    for (int j = 0; j < i; ++j) {
      const int k = f->rank[static_cast<size_t>(i) * r + j];
      const double *su = f->h_U.data() + u_src[static_cast<size_t>(i) * r + j];
      for (int c = 0; c < k; ++c, ++col)
        for (int t = 0; t < mi; ++t) {
          const double x = su[static_cast<int64_t>(t) * k + c];
          du[col * lda + t] = x;
          split_bf16(x, hi[t * kp + col], lo[t * kp + col]);
        }
    }
    // V_panel(i): row-major, columns padded to kLrRows, tiles (l, i) in
    // increasing l; the BF16 split of V_panel^T is row-major with t padded
    // to 32; zmap sends each column to its row of Z
    const int ldv = f->vpan_ld[i];
    double *dv = hv + f->vpan_off[i];
    const int64_t mp = f->vbf_mp[i];
    unsigned short *vhi = hvb + f->vbf_off[i], *vlo = vhi + f->vbf_size[i];
    col = 0;
    for (int l = i + 1; l < r; ++l) {
      const int k = f->rank[static_cast<size_t>(l) * r + i];
      const double *sv = f->h_V.data() + v_src[static_cast<size_t>(l) * r + i];
      for (int c = 0; c < k; ++c, ++col)
        for (int t = 0; t < mi; ++t) {
          const double x = sv[static_cast<int64_t>(t) * k + c];
          dv[static_cast<int64_t>(t) * ldv + col] = x;
          split_bf16(x, vhi[col * mp + t], vlo[col * mp + t]);
        }
    }
    factor_zmaps(f, i, hz + f->zmap_off[i], hzp + f->zmap_off[i]);
  }
  void **dst[8] = {reinterpret_cast<void **>(&f->d_diag), reinterpret_cast<void **>(&f->d_urow),
                   reinterpret_cast<void **>(&f->d_vpan), reinterpret_cast<void **>(&f->d_zmap),
                   reinterpret_cast<void **>(&f->d_gen),  reinterpret_cast<void **>(&f->d_ubf),
                   reinterpret_cast<void **>(&f->d_vbf),  reinterpret_cast<void **>(&f->d_zmapp)};
  int64_t total = 0;
  for (int k = 0; k < 8; ++k) {
    *dst[k] = nullptr;
    if (sizes[k] == 0) continue;
    *dst[k] = ctx->dmalloc(sizes[k]);
    if (!*dst[k]) return fail(TLRQMC_ENOMEM, "device allocation of %zu bytes failed", sizes[k]);
    total += static_cast<int64_t>(sizes[k]);
    if (hipMemcpyAsync(*dst[k], stage + offs[k], sizes[k], hipMemcpyHostToDevice, ctx->stream) != hipSuccess)
      return fail(TLRQMC_EDEVICE, "hipMemcpyAsync to device failed");
  }
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return fail(TLRQMC_EDEVICE, "stream synchronize failed");
  f->device_bytes = total;
  {
    // FNV-1a over 64-bit words (the last one zero-padded) within 1 MiB
    // chunks, hashed in parallel; the chunk hashes are folded in order.
    constexpr size_t kChunk = size_t{1} << 20;
    const std::pair<const void *, size_t> parts[5] = {{f->perm.data(), f->perm.size() * 4},
                                                      {f->h_diag.data(), f->h_diag.size() * 8},
                                                      {f->rank.data(), f->rank.size() * 4},
                                                      {f->h_U.data(), f->h_U.size() * 8},
                                                      {f->h_V.data(), f->h_V.size() * 8}};
    std::vector<std::pair<const unsigned char *, size_t>> chunks;
    for (const auto &pt : parts)
      for (size_t o = 0; o < pt.second; o += kChunk)
        chunks.push_back({static_cast<const unsigned char *>(pt.first) + o, std::min(kChunk, pt.second - o)});
    std::vector<uint64_t> ch(chunks.size());
#pragma omp parallel for schedule(dynamic, 4)
    for (size_t q = 0; q < chunks.size(); ++q) {
      uint64_t h = 1469598103934665603ull;
      const unsigned char *c = chunks[q].first;
      const size_t bytes = chunks[q].second;
      for (size_t o = 0; o < bytes; o += 8) {
        uint64_t w = 0;
        std::memcpy(&w, c + o, std::min<size_t>(8, bytes - o));
        h = (h ^ w) * 1099511628211ull;
      }
      ch[q] = h;
    }
    uint64_t hsh = 1469598103934665603ull;
    for (uint64_t h : ch) hsh = (hsh ^ h) * 1099511628211ull;
    f->checksum = hsh;
  }
  *out = guard.release();
  return TLRQMC_OK;
}

}  // namespace

int factor_build(tlrqmc_ctx *ctx, int64_t n, int m, const int32_t *perm, const double *diag,
                 const int32_t *ranks, const double *U, const double *V, int cap_hits,
                 tlrqmc_factor **out) {
  return build_impl(ctx, n, m, perm, diag, ranks, U, V, cap_hits, nullptr, nullptr, nullptr, out);
}

int factor_build_take(tlrqmc_ctx *ctx, int64_t n, int m, const int32_t *perm, std::vector<double> &diag,
                      const int32_t *ranks, std::vector<double> &U, std::vector<double> &V, int cap_hits,
                      tlrqmc_factor **out) {
  return build_impl(ctx, n, m, perm, diag.data(), ranks, U.data(), V.data(), cap_hits, &diag, &U, &V, out);
}

}  // namespace tlrqmc

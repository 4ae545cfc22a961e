// Factor construction: exchange layout on the host -> device layouts.
//
// The TLR factor of Section 3.4 is r diagonal tiles B_i and off-diagonal
// tiles L_ij = U_ij V_ij^T (i > j).  The estimator walks the tiles left
// looking: Delta_i = sum_j<i U_ij (V_ij^T y_j) = U_row(i) Z_row(i), where
// U_row(i) = [U_i0 ... U_i,i-1] and Z_row(i) stacks the rank-space images
// V_ij^T y_j.  Those images are produced right after tile j by one product
// with V_panel(j) = [V_j+1,j ... V_r-1,j]; zmap sends each of its columns
// to the row of Z_row(i) it belongs to.
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>

#include "internal.hpp"

namespace tlrqmc {

namespace {

int upload(tlrqmc_ctx *ctx, const void *host, size_t bytes, void **dev, int64_t &total) {
  *dev = nullptr;
  if (bytes == 0) return TLRQMC_OK;
  *dev = ctx->dmalloc(bytes);
  if (!*dev) return fail(TLRQMC_ENOMEM, "device allocation of %zu bytes failed", bytes);
  total += static_cast<int64_t>(bytes);
  if (hipMemcpyAsync(*dev, host, bytes, hipMemcpyHostToDevice, ctx->stream) != hipSuccess)
    return fail(TLRQMC_EDEVICE, "hipMemcpyAsync to device failed");
  return TLRQMC_OK;
}

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

int factor_build(tlrqmc_ctx *ctx, int64_t n, int m, const int32_t *perm, const double *diag,
                 const int32_t *ranks, const double *U, const double *V, int cap_hits,
                 tlrqmc_factor **out) {
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
  f->n = n;
  f->m = m;
  f->r = r;
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
  f->tm.resize(r);
  f->toff.resize(r + 1);
  for (int i = 0; i < r; ++i) {
    f->toff[i] = static_cast<int64_t>(i) * m;
    f->tm[i] = static_cast<int>(std::min<int64_t>(m, n - f->toff[i]));
  }
  f->toff[r] = n;
  // ranks and the derived widths
  f->rank.assign(static_cast<size_t>(r) * r, 0);
  f->krow.assign(r, 0);
  f->kcol.assign(r, 0);
  int64_t uv_doubles_u = 0, uv_doubles_v = 0;
  for (int i = 1; i < r; ++i)
    for (int j = 0; j < i; ++j) {
      const int k = ranks[static_cast<size_t>(i) * r + j];
      if (k < 0 || k > std::min(f->tm[i], f->tm[j]))
        return fail(TLRQMC_EINVAL, "rank of tile (%d,%d) out of range: %d", i, j, k);
      if (k > 0 && (!U || !V)) return fail(TLRQMC_EINVAL, "U and V are required for nonzero ranks");
      f->rank[static_cast<size_t>(i) * r + j] = k;
      f->krow[i] += k;
      f->kcol[j] += k;
      f->k_max = std::max(f->k_max, k);
      uv_doubles_u += static_cast<int64_t>(f->tm[i]) * k;
      uv_doubles_v += static_cast<int64_t>(f->tm[j]) * k;
    }
  f->zoff.assign(r + 1, 0);
  for (int i = 0; i < r; ++i) f->zoff[i + 1] = f->zoff[i] + f->krow[i];
  f->k_tot = f->zoff[r];
  if (f->k_tot > (int64_t{1} << 31) - 1) return fail(TLRQMC_EINVAL, "total rank too large");
  // host exchange copies (validated)
  int64_t diag_doubles = 0;
  for (int i = 0; i < r; ++i) diag_doubles += static_cast<int64_t>(f->tm[i]) * f->tm[i];
  f->h_diag.assign(diag, diag + diag_doubles);
  if (uv_doubles_u) {
    f->h_U.assign(U, U + uv_doubles_u);
    f->h_V.assign(V, V + uv_doubles_v);
  }
  {
    int64_t o = 0;
    for (int i = 0; i < r; ++i) {
      const int mi = f->tm[i];
      for (int t = 0; t < mi; ++t) {
        for (int u = 0; u <= t; ++u) {
          const double v = f->h_diag[o + static_cast<int64_t>(t) * mi + u];
          if (!std::isfinite(v)) return fail(TLRQMC_EINVAL, "non-finite diagonal-tile entry in tile %d", i);
        }
        if (!(f->h_diag[o + static_cast<int64_t>(t) * mi + t] > 0.0))
          return fail(TLRQMC_EINVAL, "diagonal entry %lld is not positive", static_cast<long long>(f->toff[i] + t));
      }
      o += static_cast<int64_t>(mi) * mi;
    }
    for (double v : f->h_U)
      if (!std::isfinite(v)) return fail(TLRQMC_EINVAL, "non-finite entry in U");
    for (double v : f->h_V)
      if (!std::isfinite(v)) return fail(TLRQMC_EINVAL, "non-finite entry in V");
  }
  // ---- blocked diagonal tiles (row blocks of SB, see the sweep kernel)
  constexpr int SB = kSweepBlock;
  std::vector<double> hb;
  f->diag_off.assign(r + 1, 0);
  {
    int64_t o = 0;
    for (int i = 0; i < r; ++i) {
      const int mi = f->tm[i];
      const int nb = (mi + SB - 1) / SB;
      f->diag_off[i] = static_cast<int64_t>(hb.size());
      hb.resize(hb.size() + static_cast<size_t>(nb) * (nb + 1) / 2 * SB * SB, 0.0);
      double *T = hb.data() + f->diag_off[i];
      const double *src = f->h_diag.data() + o;
      auto Bat = [&](int t, int u) { return src[static_cast<int64_t>(t) * mi + u]; };
      for (int q = 0; q < nb; ++q) {
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
      }
      o += static_cast<int64_t>(mi) * mi;
    }
    f->diag_off[r] = static_cast<int64_t>(hb.size());
  }
  // ---- U_row(i) column-major (rows padded to kLrRows), V_panel(j) row-major
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
  std::vector<double> hu, hv;
  std::vector<int32_t> hz;
  f->urow_off.assign(r + 1, 0);
  f->urow_ld.assign(r, 0);
  for (int i = 0; i < r; ++i) {
    const int lda = static_cast<int>(round_up(f->tm[i], kLrRows));
    f->urow_ld[i] = lda;
    f->urow_off[i] = static_cast<int64_t>(hu.size());
    hu.resize(hu.size() + static_cast<size_t>(lda) * f->krow[i], 0.0);
    double *dst = hu.data() + f->urow_off[i];
    int64_t col = 0;
    for (int j = 0; j < i; ++j) {
      const int k = f->rank[static_cast<size_t>(i) * r + j];
      const double *src = f->h_U.data() + u_src[static_cast<size_t>(i) * r + j];
      for (int c = 0; c < k; ++c, ++col)
        for (int t = 0; t < f->tm[i]; ++t) dst[col * lda + t] = src[static_cast<int64_t>(t) * k + c];
    }
  }
  f->urow_off[r] = static_cast<int64_t>(hu.size());
  f->vpan_off.assign(r + 1, 0);
  f->vpan_ld.assign(r, 0);
  f->zmap_off.assign(r + 1, 0);
  for (int j = 0; j < r; ++j) {
    const int ldv = static_cast<int>(round_up(std::max<int64_t>(f->kcol[j], 1), kLrRows));
    f->vpan_ld[j] = ldv;
    f->vpan_off[j] = static_cast<int64_t>(hv.size());
    f->zmap_off[j] = static_cast<int64_t>(hz.size());
    hv.resize(hv.size() + static_cast<size_t>(ldv) * f->tm[j], 0.0);
    double *dst = hv.data() + f->vpan_off[j];
    int64_t col = 0;
    for (int i = j + 1; i < r; ++i) {
      const int k = f->rank[static_cast<size_t>(i) * r + j];
      if (k == 0) continue;
      // Z row of (i, j, c): zoff[i] + (ranks of tiles (i, 0..j-1)) + c
      int64_t zr = f->zoff[i];
      for (int jj = 0; jj < j; ++jj) zr += f->rank[static_cast<size_t>(i) * r + jj];
      const double *src = f->h_V.data() + v_src[static_cast<size_t>(i) * r + j];
      for (int c = 0; c < k; ++c, ++col) {
        for (int t = 0; t < f->tm[j]; ++t) dst[static_cast<int64_t>(t) * ldv + col] = src[static_cast<int64_t>(t) * k + c];
        hz.push_back(static_cast<int32_t>(zr + c));
      }
    }
  }
  f->vpan_off[r] = static_cast<int64_t>(hv.size());
  f->zmap_off[r] = static_cast<int64_t>(hz.size());
  // ---- precision form: BF16 hi/lo splits and the padded Z layout
  f->kp_row.assign(r, 0);
  f->zoffp.assign(r + 1, 0);
  for (int i = 0; i < r; ++i) {
    f->kp_row[i] = static_cast<int>(round_up(f->krow[i], 32));
    f->zoffp[i + 1] = f->zoffp[i] + f->kp_row[i];
  }
  f->zp_tot = f->zoffp[r];
  std::vector<unsigned short> hub, hvb;
  std::vector<int32_t> hzp;
  f->ubf_off.assign(r + 1, 0);
  f->ubf_size.assign(r, 0);
  for (int i = 0; i < r; ++i) {
    const int64_t rows = lr_mfma_rows(f->tm[i]);
    const int64_t kp = f->kp_row[i];
    f->ubf_off[i] = static_cast<int64_t>(hub.size());
    f->ubf_size[i] = rows * kp;
    hub.resize(hub.size() + 2 * rows * kp, 0);
    unsigned short *hi = hub.data() + f->ubf_off[i], *lo = hi + rows * kp;
    const double *src = hu.data() + f->urow_off[i];  // column-major, lda = urow_ld[i]
    for (int64_t col = 0; col < f->krow[i]; ++col)
      for (int t = 0; t < f->tm[i]; ++t) split_bf16(src[col * f->urow_ld[i] + t], hi[t * kp + col], lo[t * kp + col]);
  }
  f->ubf_off[r] = static_cast<int64_t>(hub.size());
  f->vbf_off.assign(r + 1, 0);
  f->vbf_size.assign(r, 0);
  f->vbf_mp.assign(r, 0);
  for (int j = 0; j < r; ++j) {
    const int64_t kp = lr_mfma_rows(static_cast<int>(f->kcol[j]));
    const int64_t mp = round_up(f->tm[j], 32);
    f->vbf_mp[j] = static_cast<int>(mp);
    f->vbf_off[j] = static_cast<int64_t>(hvb.size());
    f->vbf_size[j] = kp * mp;
    hvb.resize(hvb.size() + 2 * kp * mp, 0);
    unsigned short *hi = hvb.data() + f->vbf_off[j], *lo = hi + kp * mp;
    const double *src = hv.data() + f->vpan_off[j];  // row-major, ldv = vpan_ld[j]
    for (int64_t col = 0; col < f->kcol[j]; ++col) {
      for (int t = 0; t < f->tm[j]; ++t) split_bf16(src[static_cast<int64_t>(t) * f->vpan_ld[j] + col], hi[col * mp + t], lo[col * mp + t]);
      // padded Z row of the same (i, j, c) as the unpadded zmap entry
      const int32_t zr = hz[f->zmap_off[j] + col];
      int i = 0;
      while (f->zoff[i + 1] <= zr) ++i;
      hzp.push_back(static_cast<int32_t>(f->zoffp[i] + (zr - f->zoff[i])));
    }
  }
  f->vbf_off[r] = static_cast<int64_t>(hvb.size());
  // lattice generators A_0..A_n
  const std::vector<uint64_t> gen = richtmyer_generators(n + 1);
  int64_t total = 0;
  int st;
  if ((st = upload(ctx, hb.data(), hb.size() * sizeof(double), reinterpret_cast<void **>(&f->d_diag), total))) return st;
  if ((st = upload(ctx, hu.data(), hu.size() * sizeof(double), reinterpret_cast<void **>(&f->d_urow), total))) return st;
  if ((st = upload(ctx, hv.data(), hv.size() * sizeof(double), reinterpret_cast<void **>(&f->d_vpan), total))) return st;
  if ((st = upload(ctx, hz.data(), hz.size() * sizeof(int32_t), reinterpret_cast<void **>(&f->d_zmap), total))) return st;
  if ((st = upload(ctx, gen.data(), gen.size() * sizeof(uint64_t), reinterpret_cast<void **>(&f->d_gen), total))) return st;
  if ((st = upload(ctx, hub.data(), hub.size() * 2, reinterpret_cast<void **>(&f->d_ubf), total))) return st;
  if ((st = upload(ctx, hvb.data(), hvb.size() * 2, reinterpret_cast<void **>(&f->d_vbf), total))) return st;
  if ((st = upload(ctx, hzp.data(), hzp.size() * 4, reinterpret_cast<void **>(&f->d_zmapp), total))) return st;
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return fail(TLRQMC_EDEVICE, "stream synchronize failed");
  f->device_bytes = total;
  *out = guard.release();
  return TLRQMC_OK;
}

}  // namespace tlrqmc

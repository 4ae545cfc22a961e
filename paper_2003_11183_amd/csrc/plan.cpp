// Host-side plan of the estimator (see plan.hpp): factor layout, chunk
// buffers and the descriptors of one tile step.
#include "plan.hpp"

#include <algorithm>

namespace tlrqmc {

void factor_geometry(tlrqmc_factor *f, int64_t n, int m, const int32_t *ranks) {
  const int r = static_cast<int>((n + m - 1) / m);
  f->n = n;
  f->m = m;
  f->r = r;
  f->tm.resize(r);
  f->toff.resize(r + 1);
  for (int i = 0; i < r; ++i) {
    f->toff[i] = static_cast<int64_t>(i) * m;
    f->tm[i] = static_cast<int>(std::min<int64_t>(m, n - f->toff[i]));
  }
  f->toff[r] = n;
  f->rank.assign(static_cast<size_t>(r) * r, 0);
  f->krow.assign(r, 0);
  f->kcol.assign(r, 0);
  f->k_max = 0;
  for (int i = 1; i < r; ++i)
    for (int j = 0; j < i; ++j) {
      const int k = ranks[static_cast<size_t>(i) * r + j];
      f->rank[static_cast<size_t>(i) * r + j] = k;
      f->krow[i] += k;
      f->kcol[j] += k;
      f->k_max = std::max(f->k_max, k);
    }
  f->zoff.assign(r + 1, 0);
  for (int i = 0; i < r; ++i) f->zoff[i + 1] = f->zoff[i] + f->krow[i];
  f->k_tot = f->zoff[r];
}

void factor_layout(tlrqmc_factor *f) {
  const int r = f->r;
  constexpr int SB = kSweepBlock;
  f->diag_off.assign(r + 1, 0);
  f->urow_off.assign(r + 1, 0);
  f->urow_ld.assign(r, 0);
  f->vpan_off.assign(r + 1, 0);
  f->vpan_ld.assign(r, 0);
  f->zmap_off.assign(r + 1, 0);
  f->kp_row.assign(r, 0);
  f->zoffp.assign(r + 1, 0);
  f->ubf_off.assign(r + 1, 0);
  f->ubf_size.assign(r, 0);
  f->vbf_off.assign(r + 1, 0);
  f->vbf_size.assign(r, 0);
  f->vbf_mp.assign(r, 0);
  for (int i = 0; i < r; ++i) {
    // blocked diagonal tile: row block q holds blocks (q, 0..q)
    const int nb = (f->tm[i] + SB - 1) / SB;
    f->diag_off[i + 1] = f->diag_off[i] + static_cast<int64_t>(nb) * (nb + 1) / 2 * SB * SB;
    f->urow_ld[i] = static_cast<int>(round_up(f->tm[i], kLrRows));
    f->urow_off[i + 1] = f->urow_off[i] + static_cast<int64_t>(f->urow_ld[i]) * f->krow[i];
    f->vpan_ld[i] = static_cast<int>(round_up(std::max<int64_t>(f->kcol[i], 1), kLrRows));
    f->vpan_off[i + 1] = f->vpan_off[i] + static_cast<int64_t>(f->vpan_ld[i]) * f->tm[i];
    f->zmap_off[i + 1] = f->zmap_off[i] + f->kcol[i];
    // precision form: BF16 hi/lo splits and a Z layout with row blocks padded to 32
    f->kp_row[i] = static_cast<int>(round_up(f->krow[i], 32));
    f->zoffp[i + 1] = f->zoffp[i] + f->kp_row[i];
    f->ubf_size[i] = lr_mfma_rows(f->tm[i]) * f->kp_row[i];
    f->ubf_off[i + 1] = f->ubf_off[i] + 2 * f->ubf_size[i];
    f->vbf_mp[i] = static_cast<int>(round_up(f->tm[i], 32));
    f->vbf_size[i] = lr_mfma_rows(static_cast<int>(f->kcol[i])) * f->vbf_mp[i];
    f->vbf_off[i + 1] = f->vbf_off[i] + 2 * f->vbf_size[i];
  }
  f->zp_tot = f->zoffp[r];
}

void factor_device_sizes(const tlrqmc_factor *f, size_t sizes[8]) {
  const int r = f->r;
  sizes[0] = static_cast<size_t>(f->diag_off[r]) * 8;
  sizes[1] = static_cast<size_t>(f->urow_off[r]) * 8;
  sizes[2] = static_cast<size_t>(f->vpan_off[r]) * 8;
  sizes[3] = static_cast<size_t>(f->zmap_off[r]) * 4;
  sizes[4] = static_cast<size_t>(f->n + 1) * 8;
  sizes[5] = static_cast<size_t>(f->ubf_off[r]) * 2;
  sizes[6] = static_cast<size_t>(f->vbf_off[r]) * 2;
  sizes[7] = static_cast<size_t>(f->zmap_off[r]) * 4;
}

// Column c of tile (l, i) in V_panel(i) feeds row l of the recursion: its
// image lands in Z_row(l) after the images of tiles (l, 0..i-1).
void factor_zmaps(const tlrqmc_factor *f, int i, int32_t *z, int32_t *zp) {
  const int r = f->r;
  int64_t col = 0;
  for (int l = i + 1; l < r; ++l) {
    const int k = f->rank[static_cast<size_t>(l) * r + i];
    if (k == 0) continue;
    int64_t zr = f->zoff[l];
    for (int jj = 0; jj < i; ++jj) zr += f->rank[static_cast<size_t>(l) * r + jj];
    for (int c = 0; c < k; ++c, ++col) {
      z[col] = static_cast<int32_t>(zr + c);
      zp[col] = static_cast<int32_t>(f->zoffp[l] + (zr + c - f->zoff[l]));
    }
  }
}

void chunk_buffer_bytes(const tlrqmc_factor *f, bool prec, bool scaled, int64_t ld, int64_t bytes[4]) {
  const int64_t mpad = round_up(f->m, 64);
  const int64_t w = prec ? 4 : 8;
  bytes[0] = w * mpad * ld;
  bytes[1] = f->r > 1 ? w * mpad * ld : 0;
  bytes[2] = f->k_tot > 0 ? (prec ? 4 * f->zp_tot * ld : 8 * f->k_tot * ld) : 0;
  bytes[3] = scaled ? 8 * ld : 0;
}

int64_t chunk_bytes_per_sample(const tlrqmc_factor *f, bool prec) {
  const int64_t mpad = round_up(f->m, 64);
  return prec ? 4 * f->zp_tot + 8 * mpad + 16 : 8 * (f->k_tot + 2 * mpad + 2);
}

int64_t estimator_call_bytes(int64_t n, int M, int64_t count, bool two_sided, bool reduce) {
  return (two_sided ? round_up(8 * n, 256) : 0) + round_up(8 * n, 256) +
         round_up(8 * static_cast<int64_t>(M) * (n + 1), 256) + round_up(8 * count, 256) +
         (reduce ? round_up(8 * 3 * M, 256) : 0);
}

ChunkPlan plan_chunks(const tlrqmc_factor *f, bool prec, int64_t count, int64_t requested, int64_t fixed_left,
                      int64_t call_bytes) {
  const int64_t per_sample = chunk_bytes_per_sample(f, prec);
  const bool fixed = fixed_left >= 0;
  ChunkPlan p{(!fixed && count >= kMultiStreamSamples) ? kWorkerStreams : 1, requested};
  if (fixed) {
    // what is left of the region after the per-call arrays, in chunks of 256
    // (slack for the rounding of the four chunk buffers and one more)
    const int64_t room = fixed_left - call_bytes - 5 * 256;
    const int64_t fit = room > 0 ? room / per_sample / 256 * 256 : 0;
    if (fit < 256) return ChunkPlan{1, 0};
    p.chunk = p.chunk > 0 ? std::min(p.chunk, fit) : fit;
  } else if (p.chunk <= 0) {
    const int64_t budget = kScratchBudget / p.nstream;
    p.chunk = std::max<int64_t>(256, std::min<int64_t>(budget / per_sample, (count + p.nstream - 1) / p.nstream));
  }
  p.chunk = round_up(std::min({p.chunk, count, kMaxChunk}), 256);
  return p;
}

SlotPlan plan_slots(const tlrqmc_factor *f, bool prec, bool scaled, int64_t count) {
  auto slot_bytes = [&](int64_t ld) {
    int64_t b[4], sum = 0;
    chunk_buffer_bytes(f, prec, scaled, ld, b);
    for (int k = 0; k < 4; ++k) sum += round_up(b[k], 256);
    return sum;
  };
  const int64_t per_sample = slot_bytes(256) / 256 + 1;
  const int64_t chunk = std::min<int64_t>({count, kSlotSamples, std::max<int64_t>(256, kSlotBytes / per_sample)});
  const int64_t nslots = (count + chunk - 1) / chunk;
  SlotPlan p;
  p.chunk = round_up((count + nslots - 1) / nslots, 256);
  p.nslots = static_cast<int>((count + p.chunk - 1) / p.chunk);
  p.slot_bytes = slot_bytes(p.chunk);
  return p;
}

InitParams init_launch(const tlrqmc_factor *f, const ChunkRun &c, double nu) {
  return InitParams{c.g0, c.count, c.N, f->d_gen, c.D, f->n + 1, nu, c.logp, c.buf.R};
}

TileLaunch tile_launch(const tlrqmc_factor *f, int j, const ChunkRun &c) {
  TileLaunch t;
  const ChunkBuffers &L = c.buf;
  const int64_t ld = c.ld;
  t.delta = j > 0 && f->krow[j] > 0;
  if (t.delta) {
    if (c.prec) {
      const unsigned short *u = f->d_ubf + f->ubf_off[j];
      t.delta_mfma = MfmaLrParams{c.count, ld, f->tm[j], static_cast<int>(f->krow[j]), f->kp_row[j], u,
                                  u + f->ubf_size[j], L.ZF + f->zoffp[j] * ld, nullptr, nullptr, L.DlF};
    } else {
      t.delta_f64 = LrParams{c.count, ld, f->tm[j], static_cast<int>(f->krow[j]), f->urow_ld[j],
                             f->d_urow + f->urow_off[j], L.Z + f->zoff[j] * ld, L.Dl, nullptr};
    }
  }
  const void *delta = t.delta ? (c.prec ? static_cast<const void *>(L.DlF) : static_cast<const void *>(L.Dl)) : nullptr;
  t.sweep = SweepParams{c.g0, c.count, c.N, ld, f->n + 1, f->tm[j], static_cast<int>(1 + f->toff[j]),
                        f->d_diag + f->diag_off[j], c.a ? c.a + f->toff[j] : nullptr, c.b + f->toff[j],
                        delta, L.R, f->d_gen, c.D, c.logp, L.Y};
  t.zproj = j < f->r - 1 && f->kcol[j] > 0;
  if (t.zproj) {
    if (c.prec) {
      const unsigned short *v = f->d_vbf + f->vbf_off[j];
      t.zproj_mfma = MfmaLrParams{c.count, ld, static_cast<int>(f->kcol[j]), f->tm[j], f->vbf_mp[j], v,
                                  v + f->vbf_size[j], static_cast<const float *>(L.Y), nullptr,
                                  f->d_zmapp + f->zmap_off[j], L.ZF};
    } else {
      t.zproj_f64 = LrParams{c.count, ld, static_cast<int>(f->kcol[j]), f->tm[j], f->vpan_ld[j],
                             f->d_vpan + f->vpan_off[j], static_cast<const double *>(L.Y), L.Z,
                             f->d_zmap + f->zmap_off[j]};
    }
  }
  return t;
}

}  // namespace tlrqmc

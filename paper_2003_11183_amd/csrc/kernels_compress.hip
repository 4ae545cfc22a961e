// Compression of the off-diagonal tiles of the dense Cholesky factor on the
// device (Section 3.3: each tile L_ij is replaced by U_ij V_ij^T, keeping the
// singular values above the tolerance).  One work-group per tile, three
// passes over a batch of tiles taken in row order (tile (i, j), j < i, is
// number i (i - 1) / 2 + j):
//   k_cmp_qr  : column-pivoted Householder QR of a working copy of the tile,
//               stopped once the trailing columns' Frobenius norm is below
//               tol / 1000 (at most kCmpKq steps; a tile needing more is
//               flagged and compressed on the host);
//   k_cmp_eig : M = R R^T (kq x kq) and its eigen-decomposition M = J L J^T
//               by parallel cyclic Jacobi rotations in LDS; the singular
//               values of R are sqrt(L); the kept right vectors
//               V = R^T J_k sigma_k^-1 go to a per-tile buffer;
//   k_cmp_u   : U = T V from the untouched tile (so U V^T is T projected on
//               the kept right singular subspace), then U and V are packed
//               back to back in tile order (prefix sums over the batch).
// All arithmetic is FP64 and every reduction runs in a fixed order, so the
// factor is the same bit for bit from run to run.
#include "device_math.hpp"
#include "internal.hpp"
#include "setup_kernels.hpp"

namespace tlrqmc {

using namespace dev;

namespace {

constexpr int KQ = kCmpKq;
constexpr int MT = kCmpMaxTile;
constexpr int RPL = MT / 64;  // rows per lane of a column
constexpr int KP = KQ + 1;    // padded LDS row of M and J

struct TileAt {
  int64_t row0, col0;
  int mi, mj;
};

// Tile number t of the row order (j < i): t = i (i - 1) / 2 + j.
__device__ __host__ inline TileAt tile_at(int64_t t, int64_t n, int m) {
  int64_t i = static_cast<int64_t>((1.0 + sqrt(1.0 + 8.0 * static_cast<double>(t))) * 0.5);
  while (i * (i - 1) / 2 > t) --i;
  while ((i + 1) * i / 2 <= t) ++i;
  const int64_t j = t - i * (i - 1) / 2;
  TileAt a;
  a.row0 = i * m;
  a.col0 = j * m;
  a.mi = static_cast<int>(n - a.row0 < m ? n - a.row0 : m);
  a.mj = static_cast<int>(n - a.col0 < m ? n - a.col0 : m);
  return a;
}

// DPP move of a double (both halves); lanes whose source is outside the
// pattern or masked off read 0.
template <int CTRL, int ROW_MASK = 0xf>
__device__ inline double dpp_mov(double x) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(u & 0xffffffffu), CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(u >> 32), CTRL, ROW_MASK, 0xf, false);
  return __builtin_bit_cast(double, (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) |
                                        static_cast<uint32_t>(lo));
}

// Sum over the wave with DPP (no LDS traffic): sums within rows of 16 lanes
// by row shifts 1, 2, 4, 8, then row broadcasts 15 and 31 carry the rows'
// totals up; lane 63 holds the total, which every lane gets.
__device__ inline double wave_sum(double v) {
  v += dpp_mov<0x111>(v);        // row_shr:1
  v += dpp_mov<0x112>(v);        // row_shr:2
  v += dpp_mov<0x114>(v);        // row_shr:4
  v += dpp_mov<0x118>(v);        // row_shr:8
  v += dpp_mov<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_mov<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(u & 0xffffffffu), 63));
  const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(u >> 32), 63));
  return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

__device__ inline int64_t wave_sum_i64(int64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// ------------------------------------------------------------------- QR pass
// Working copy W (column-major, leading dimension mi) of the mi x mj tile.
// Step k picks the unselected column of largest trailing norm (lowest index
// on ties), reflects rows k.. of every unselected column with the Householder
// vector of that column and recomputes their trailing norms.  The selected
// column keeps its R entries (rows 0..k) and is zeroed below.  On exit rows
// 0..kq-1 of W hold R with its columns in the tile's own order.
__global__ __launch_bounds__(256) void k_cmp_qr(const double *L, int64_t lda, int64_t n, int m, int64_t t0,
                                                double tol, double *W, int64_t wslot, int32_t *info) {
  __shared__ double cn[MT];
  __shared__ double vb[MT];
  __shared__ int sel[MT];
  __shared__ double red_v[4], red_s[4];
  __shared__ int red_i[4];
  __shared__ double s_tau;
  const int s = static_cast<int>(blockIdx.x);
  const TileAt tl = tile_at(t0 + s, n, m);
  const int mi = tl.mi, mj = tl.mj;
  const int tid = static_cast<int>(threadIdx.x), w = tid >> 6, lane = tid & 63;
  double *Ws = W + static_cast<int64_t>(s) * wslot;
  const double *T = L + tl.col0 * lda + tl.row0;
  const int nq = (mi + 63) >> 6;
  for (int c = w; c < mj; c += 4) {
    double ss = 0.0;
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int r = lane + 64 * q;
      if (q < nq && r < mi) {
        const double x = T[c * lda + r];
        Ws[c * mi + r] = x;
        ss = fma(x, x, ss);
      }
    }
    ss = wave_sum(ss);
    if (lane == 0) cn[c] = ss;
  }
  for (int c = tid; c < mj; c += 256) sel[c] = 0;
  const double stop = 1e-3 * tol, stop2 = stop * stop;
  const int kmax = min(mi, mj);
  int kq = 0, flags = 0;
  for (;; ++kq) {
    __syncthreads();
    double bv = -1.0, sum = 0.0;
    int bi = MT;
    for (int c = tid; c < mj; c += 256)
      if (!sel[c]) {
        const double x = cn[c];
        sum += x;
        if (x > bv) {
          bv = x;
          bi = c;
        }
      }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(bv, o);
      const int oi = __shfl_xor(bi, o);
      if (ov > bv || (ov == bv && oi < bi)) {
        bv = ov;
        bi = oi;
      }
    }
    sum = wave_sum(sum);
    if (lane == 0) {
      red_v[w] = bv;
      red_i[w] = bi;
      red_s[w] = sum;
    }
    __syncthreads();
    const double rest = ((red_s[0] + red_s[1]) + red_s[2]) + red_s[3];
    double pv = red_v[0];
    int p = red_i[0];
    for (int u = 1; u < 4; ++u)
      if (red_v[u] > pv || (red_v[u] == pv && red_i[u] < p)) {
        pv = red_v[u];
        p = red_i[u];
      }
    if (kq >= kmax || !(rest > stop2) || p >= mj) break;
    if (kq == KQ) {
      flags |= 1;  // more than KQ steps needed: left to the host
      break;
    }
    // Householder vector of column p, rows kq..mi-1 (wave 0)
    if (w == 0) {
      double x[RPL];
      double n2 = 0.0, t2 = 0.0;
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        const int r = lane + 64 * q;
        x[q] = (q < nq && r >= kq && r < mi) ? Ws[p * mi + r] : 0.0;
        n2 = fma(x[q], x[q], n2);
        if (r > kq) t2 = fma(x[q], x[q], t2);
      }
      n2 = wave_sum(n2);
      t2 = wave_sum(t2);
      const double xk = Ws[p * mi + kq];
      const double nrm = sqrt(n2);
      const double alpha = xk >= 0.0 ? -nrm : nrm;
      const double v0 = xk - alpha;
      const double vn2 = fma(v0, v0, t2);
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        const int r = lane + 64 * q;
        if (q < nq && r >= kq && r < mi) {
          vb[r] = r == kq ? v0 : x[q];
          Ws[p * mi + r] = r == kq ? alpha : 0.0;
        }
      }
      if (lane == 0) {
        s_tau = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
        sel[p] = 1;
      }
    }
    __syncthreads();
    const double tau = s_tau;
    for (int c = w; c < mj; c += 4) {
      if (sel[c]) continue;
      double x[RPL];
      double d = 0.0;
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        const int r = lane + 64 * q;
        x[q] = (q < nq && r >= kq && r < mi) ? Ws[c * mi + r] : 0.0;
        d = fma(r < mi && r >= kq ? vb[r] : 0.0, x[q], d);
      }
      d = wave_sum(d) * tau;
      double t2 = 0.0;
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        const int r = lane + 64 * q;
        if (q < nq && r >= kq && r < mi) {
          x[q] = fma(-d, vb[r], x[q]);
          Ws[c * mi + r] = x[q];
          if (r > kq) t2 = fma(x[q], x[q], t2);
        }
      }
      t2 = wave_sum(t2);
      if (lane == 0) cn[c] = t2;
    }
  }
  if (tid == 0) {
    info[4 * s + 0] = kq;
    info[4 * s + 1] = 0;
    info[4 * s + 2] = flags;
  }
}

// ---------------------------------------------------------------- eigen pass
// Circle-method pairing of the players 0..ne-1: slot 0 keeps player 0, the
// other slots rotate by one each round; round t pairs slots i and ne-1-i.
__device__ inline int player(int slot, int round, int ne) {
  return slot == 0 ? 0 : 1 + (slot - 1 + round) % (ne - 1);
}

__global__ __launch_bounds__(256) void k_cmp_eig(const double *W, int64_t wslot, int64_t n, int m, int64_t t0,
                                                 double tol, int cap, double *Vs, int64_t vslot, int32_t *info) {
  __shared__ double Ms[KQ * KP];
  __shared__ double Js[KQ * KP];
  __shared__ int pp[KQ / 2], pq[KQ / 2];
  __shared__ double pc[KQ / 2], ps[KQ / 2];
  __shared__ double sig[KQ];
  __shared__ int ord[KQ];
  __shared__ double red[4];
  const int s = static_cast<int>(blockIdx.x);
  const int kq = info[4 * s + 0], flags = info[4 * s + 2];
  if ((flags & 1) || kq == 0) return;  // uniform over the group
  const TileAt tl = tile_at(t0 + s, n, m);
  const int mi = tl.mi, mj = tl.mj;
  const int tid = static_cast<int>(threadIdx.x), w = tid >> 6, lane = tid & 63;
  const double *R = W + static_cast<int64_t>(s) * wslot;  // R(l, c) = R[c * mi + l]

  // M = R R^T over the padded 96 x 96 index range: thread (bp, bq) owns the
  // 6 x 6 block at rows 6 bp, columns 6 bq; R goes through LDS 64 columns at
  // a time (staged in the J area, Rc[c * KP + l]).
  {
    const int bp = tid >> 4, bq = tid & 15;
    double acc[6][6];
#pragma unroll
    for (int u = 0; u < 6; ++u)
#pragma unroll
      for (int v = 0; v < 6; ++v) acc[u][v] = 0.0;
    double *Rc = Js;
    for (int c0 = 0; c0 < mj; c0 += 64) {
      const int cw = min(64, mj - c0);
      __syncthreads();
      for (int e = tid; e < 64 * KQ; e += 256) {
        const int cc = e / KQ, l = e - cc * KQ;
        Rc[cc * KP + l] = (cc < cw && l < kq) ? R[static_cast<int64_t>(c0 + cc) * mi + l] : 0.0;
      }
      __syncthreads();
      for (int cc = 0; cc < cw; ++cc) {
        double a[6], b[6];
#pragma unroll
        for (int u = 0; u < 6; ++u) {
          a[u] = Rc[cc * KP + bp * 6 + u];
          b[u] = Rc[cc * KP + bq * 6 + u];
        }
#pragma unroll
        for (int u = 0; u < 6; ++u)
#pragma unroll
          for (int v = 0; v < 6; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 6; ++u)
#pragma unroll
      for (int v = 0; v < 6; ++v) Ms[(bp * 6 + u) * KP + bq * 6 + v] = acc[u][v];
    for (int e = tid; e < KQ * KP; e += 256) {
      const int rr = e / KP, cc = e - rr * KP;
      Js[e] = (rr == cc && rr < kq) ? 1.0 : 0.0;
    }
    __syncthreads();
  }

  // Parallel cyclic Jacobi: each round rotates ne/2 disjoint pairs at once
  // (columns of M and J, then rows of M); a sweep is ne-1 rounds.  A pair is
  // rotated unless |M_pq| is negligible against sqrt(M_pp M_qq): R is graded
  // by the pivoting, and the relative test keeps small singular values
  // accurate too.
  const int ne = kq + (kq & 1), np = ne / 2;
  if (kq >= 2) {
    for (int sweep = 0; sweep < 60; ++sweep) {
      double off = 0.0;
      for (int round = 0; round < ne - 1; ++round) {
        if (tid < np) {
          const int a = player(tid, round, ne), b = player(ne - 1 - tid, round, ne);
          const int p = min(a, b), q = max(a, b);
          double cs = 1.0, sn = 0.0;
          if (q < kq) {
            const double apq = Ms[p * KP + q];
            const double rel = sqrt(Ms[p * KP + p] * Ms[q * KP + q]);
            if (fabs(apq) > 1e-17 * rel) {
              off = fmax(off, fabs(apq) / rel);
              const double theta = (Ms[q * KP + q] - Ms[p * KP + p]) / (2.0 * apq);
              const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
              cs = 1.0 / sqrt(1.0 + t * t);
              sn = t * cs;
            }
          }
          pp[tid] = p;
          pq[tid] = q;
          pc[tid] = cs;
          ps[tid] = sn;
        }
        __syncthreads();
        for (int e = tid; e < np * kq; e += 256) {
          const int pr = e / kq, rr = e - pr * kq;
          const double sn = ps[pr];
          if (sn == 0.0) continue;
          const double cs = pc[pr];
          const int p = pp[pr], q = pq[pr];
          const double mp = Ms[rr * KP + p], mq = Ms[rr * KP + q];
          Ms[rr * KP + p] = cs * mp - sn * mq;
          Ms[rr * KP + q] = sn * mp + cs * mq;
          const double jp = Js[rr * KP + p], jq = Js[rr * KP + q];
          Js[rr * KP + p] = cs * jp - sn * jq;
          Js[rr * KP + q] = sn * jp + cs * jq;
        }
        __syncthreads();
        for (int e = tid; e < np * kq; e += 256) {
          const int pr = e / kq, cc = e - pr * kq;
          const double sn = ps[pr];
          if (sn == 0.0) continue;
          const double cs = pc[pr];
          const int p = pp[pr], q = pq[pr];
          const double mp = Ms[p * KP + cc], mq = Ms[q * KP + cc];
          Ms[p * KP + cc] = cs * mp - sn * mq;
          Ms[q * KP + cc] = sn * mp + cs * mq;
        }
        __syncthreads();
      }
      off = wave_max(off);
      if (lane == 0) red[w] = off;
      __syncthreads();
      const double all = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
      __syncthreads();
      if (all < 1e-17) break;
    }
  }

  // singular values, their descending order (lowest index on ties), rank
  for (int c = tid; c < kq; c += 256) sig[c] = sqrt(fmax(Ms[c * KP + c], 0.0));
  __syncthreads();
  for (int c = tid; c < kq; c += 256) {
    int pos = 0;
    for (int d = 0; d < kq; ++d) pos += (sig[d] > sig[c] || (sig[d] == sig[c] && d < c)) ? 1 : 0;
    ord[pos] = c;
  }
  __syncthreads();
  int k = 0;
  while (k < kq && sig[ord[k]] > tol) ++k;
  int capped = 0;
  if (cap > 0 && k > cap) {
    k = cap;
    capped = 2;
  }
  // S[l][i] = J[l][ord[i]] / sigma_ord[i] in the M area
  for (int e = tid; e < kq * k; e += 256) {
    const int l = e / k, i = e - l * k;
    Ms[l * KP + i] = Js[l * KP + ord[i]] / sig[ord[i]];
  }
  __syncthreads();
  // V (mj x k, row-major): V[c][i] = sum_l R(l, c) S[l][i], 16 columns a pass
  double *V = Vs + static_cast<int64_t>(s) * vslot;
  for (int c = tid; c < mj; c += 256)
    for (int i0 = 0; i0 < k; i0 += 16) {
      double a[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) a[u] = 0.0;
      for (int l = 0; l < kq; ++l) {
        const double rv = R[static_cast<int64_t>(c) * mi + l];
#pragma unroll
        for (int u = 0; u < 16; ++u) a[u] = fma(rv, Ms[l * KP + min(i0 + u, KQ - 1)], a[u]);
      }
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (i0 + u < k) V[static_cast<int64_t>(c) * k + i0 + u] = a[u];
    }
  if (tid == 0) {
    info[4 * s + 1] = k;
    info[4 * s + 2] = flags | capped;
  }
}

// ------------------------------------------------------- U and packing pass
// out = [U of every tile of the batch in order][V of every tile in order];
// U (mi x k) and V (mj x k) row-major.
__global__ __launch_bounds__(256) void k_cmp_u(const double *L, int64_t lda, int64_t n, int m, int64_t t0,
                                               int count, const double *Vs, int64_t vslot, const int32_t *info,
                                               double *out) {
  __shared__ int64_t red[3][4];
  const int s = static_cast<int>(blockIdx.x);
  const int tid = static_cast<int>(threadIdx.x), w = tid >> 6, lane = tid & 63;
  int64_t up = 0, vp = 0, ut = 0;
  for (int q = tid; q < count; q += 256) {
    const TileAt a = tile_at(t0 + q, n, m);
    const int64_t kk = (info[4 * q + 2] & 1) ? 0 : info[4 * q + 1];
    ut += a.mi * kk;
    if (q < s) {
      up += a.mi * kk;
      vp += a.mj * kk;
    }
  }
  up = wave_sum_i64(up);
  vp = wave_sum_i64(vp);
  ut = wave_sum_i64(ut);
  if (lane == 0) {
    red[0][w] = up;
    red[1][w] = vp;
    red[2][w] = ut;
  }
  __syncthreads();
  up = red[0][0] + red[0][1] + red[0][2] + red[0][3];
  vp = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  ut = red[2][0] + red[2][1] + red[2][2] + red[2][3];
  const int k = (info[4 * s + 2] & 1) ? 0 : info[4 * s + 1];
  if (k == 0) return;
  const TileAt tl = tile_at(t0 + s, n, m);
  const int mi = tl.mi, mj = tl.mj;
  const double *Vsrc = Vs + static_cast<int64_t>(s) * vslot;
  double *U = out + up;
  double *V = out + ut + vp;
  for (int e = tid; e < mj * k; e += 256) V[e] = Vsrc[e];
  const double *T = L + tl.col0 * lda + tl.row0;
  for (int rr = tid; rr < mi; rr += 256)
    for (int i0 = 0; i0 < k; i0 += 16) {
      double a[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) a[u] = 0.0;
      for (int c = 0; c < mj; ++c) {
        const double t = T[c * lda + rr];
#pragma unroll
        for (int u = 0; u < 16; ++u) a[u] = fma(t, i0 + u < k ? Vsrc[c * k + i0 + u] : 0.0, a[u]);
      }
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (i0 + u < k) U[static_cast<int64_t>(rr) * k + i0 + u] = a[u];
    }
}

}  // namespace

void compress_tile_at(int64_t t, int64_t n, int m, int64_t &row0, int64_t &col0, int &mi, int &mj) {
  const TileAt a = tile_at(t, n, m);
  row0 = a.row0;
  col0 = a.col0;
  mi = a.mi;
  mj = a.mj;
}

void launch_compress(hipStream_t s, const double *L, int64_t lda, int64_t n, int m, int64_t t0, int count,
                     double tol, int cap, double *W, double *Vs, double *out, int32_t *info) {
  const int64_t wslot = static_cast<int64_t>(m) * m, vslot = compress_vslot(m);
  hipLaunchKernelGGL(k_cmp_qr, dim3(count), dim3(256), 0, s, L, lda, n, m, t0, tol, W, wslot, info);
  hipLaunchKernelGGL(k_cmp_eig, dim3(count), dim3(256), 0, s, W, wslot, n, m, t0, tol, cap, Vs, vslot, info);
  hipLaunchKernelGGL(k_cmp_u, dim3(count), dim3(256), 0, s, L, lda, n, m, t0, count, Vs, vslot, info, out);
}

}  // namespace tlrqmc

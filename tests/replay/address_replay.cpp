// Address replay of the estimator's device kernels, on the host.
//
// Test infrastructure, no GPU.  The launches of an estimator call, and of
// the request server's batched steps, are built by the library's own host
// plan (csrc/plan.cpp: factor layout and row maps, chunking and slot
// sizing, per-tile descriptors, grids) over a synthetic device address
// space with one region per allocation, 1 TiB apart.  Every global load and
// store the kernels would make is recomputed from the descriptor, the grid
// and the thread index, with the kernels' own index expressions, guards and
// integer widths, and checked to lie inside the allocation its base
// pointer belongs to; the factor's per-tile operands must also stay inside
// their tile's segment.  Row maps are read from the values the factor
// build writes (factor_zmaps).
//
// Two modes.  Literal: every thread of every work-group and every loop
// value (small problems that still cover every form, ragged tiles and rank
// profile).  Extremes (full-size problems): each address is an increasing
// affine function of the sample index and of the loop counters of a
// reduction, with the row index (through a row map where there is one)
// entering as an offset, so the first and last values of each such counter
// bound every address in between; the replay visits the threads at the two
// ends of the sample range (the sweep: the first and the last live waves,
// with the dead lanes of the latter), the ends of each reduction loop, and
// every row, row block and map entry.  In both modes the work-group
// remapping of the BF16 kernel is checked to be a bijection onto its
// blocks and 32-bit offsets are checked against their 64-bit values.
//
// Usage: address_replay [name-prefix...]   Exit status 0 when every access
// lies inside its allocation.
#include <algorithm>
#include <cinttypes>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <map>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "plan.hpp"

using namespace tlrqmc;

namespace {

// ------------------------------------------------------------ address space
struct Space {
  struct Region {
    std::string name;
    uint64_t base, bytes;
  };
  std::vector<Region> regions;
  uint64_t checks = 0;
  int64_t failures = 0;
  std::string context;  // case, launch and tile being replayed

  static constexpr int kShift = 40;
  void *alloc(const std::string &name, int64_t bytes) {
    if (bytes <= 0) return nullptr;
    const uint64_t base = static_cast<uint64_t>(regions.size() + 1) << kShift;
    regions.push_back({name, base, static_cast<uint64_t>(bytes)});
    return reinterpret_cast<void *>(base);
  }
  const Region *of(uint64_t addr) const {
    const uint64_t i = addr >> kShift;
    if (i == 0 || i > regions.size()) return nullptr;
    return &regions[i - 1];
  }
  void fail(const std::string &what, uint64_t addr, uint64_t size, const std::string &why) {
    if (failures < 20)
      std::fprintf(stderr, "FAIL %s: %s [%#" PRIx64 ", +%" PRIu64 ") %s\n", context.c_str(), what.c_str(), addr, size,
                   why.c_str());
    ++failures;
  }
  // [addr, addr + size) inside the allocation that holds `from`
  void check(const void *from, uint64_t addr, uint64_t size, const char *what) {
    ++checks;
    const Region *r = of(reinterpret_cast<uint64_t>(from));
    if (!r) return fail(what, addr, size, "(base pointer outside every allocation)");
    if (addr < r->base || addr + size > r->base + r->bytes || addr + size < addr)
      return fail(what, addr, size, "outside " + r->name);
  }
  // ... and inside [seg, seg + seg_bytes)
  void check_seg(const void *seg, int64_t seg_bytes, uint64_t addr, uint64_t size, const char *what) {
    check(seg, addr, size, what);
    const uint64_t s = reinterpret_cast<uint64_t>(seg);
    if (addr < s || addr + size > s + static_cast<uint64_t>(seg_bytes)) fail(what, addr, size, "(outside the tile's segment)");
  }
};

Space S;
bool literal = false;

template <class T>
uint64_t at(const T *p, int64_t i) {
  return reinterpret_cast<uint64_t>(p) + static_cast<uint64_t>(i * static_cast<int64_t>(sizeof(T)));
}
uint64_t at_bytes(const void *p, int64_t bytes) { return reinterpret_cast<uint64_t>(p) + static_cast<uint64_t>(bytes); }

// Values of a counter in [lo, hi) that the replay visits.
std::vector<int64_t> span(int64_t lo, int64_t hi) {
  std::vector<int64_t> v;
  if (hi <= lo) return v;
  if (literal || hi - lo <= 2) {
    for (int64_t x = lo; x < hi; ++x) v.push_back(x);
  } else {
    v = {lo, hi - 1};
  }
  return v;
}
// Members of a set of candidates inside [0, n), each once.
std::vector<int64_t> within(std::initializer_list<int64_t> c, int64_t n) {
  std::vector<int64_t> v;
  for (int64_t x : c)
    if (x >= 0 && x < n && std::find(v.begin(), v.end(), x) == v.end()) v.push_back(x);
  std::sort(v.begin(), v.end());
  return v;
}

// Row maps: device address of a map array -> the host values written there.
std::map<uint64_t, const int32_t *> g_maps;
int64_t map_value(const int32_t *map, int64_t i) {
  const Space::Region *r = S.of(reinterpret_cast<uint64_t>(map));
  auto it = r ? g_maps.find(r->base) : g_maps.end();
  if (it == g_maps.end()) {
    S.fail("map", reinterpret_cast<uint64_t>(map), 4, "(no host copy of the map)");
    return 0;
  }
  return it->second[(reinterpret_cast<uint64_t>(map) - r->base) / 4 + i];
}

// Work already replayed whose addresses do not depend on the chunk (factor
// operands of a tile): done once per call.
std::set<std::tuple<uint64_t, int64_t, int64_t, int64_t>> g_done;
bool first_time(const void *p, int64_t a, int64_t b, int64_t c) {
  return g_done.insert({reinterpret_cast<uint64_t>(p), a, b, c}).second;
}

// Low-rank launches with a descriptor already replayed in this call (the
// same chunk buffers and sample count in a later chunk) make the same
// accesses: replayed once.
std::set<std::string> g_seen;
template <class P>
bool new_descriptor(const P &p) {
  return g_seen.insert(std::string(reinterpret_cast<const char *>(&p), sizeof p)).second;
}

// Threads (one sample each) replayed along a launch of nthreads threads
// whose samples end at count.
std::vector<int64_t> sample_threads(int64_t nthreads, int64_t count) {
  if (literal) {
    std::vector<int64_t> v;
    for (int64_t i = 0; i < nthreads; ++i) v.push_back(i);
    return v;
  }
  return within({0, 1, count - 2, count - 1, count, nthreads - 1}, nthreads);
}

// ------------------------------------------------------------------- init
void replay_init(const InitParams &p, Grid g) {
  for (int64_t i : sample_threads(static_cast<int64_t>(g.x) * 256, p.count)) {
    if (i >= p.count) continue;
    S.check(p.logp, at(p.logp, i), 8, "init logp");
    if (p.nu > 0.0) {
      const int64_t s = (p.g0 + i) / p.N;
      S.check(p.A, at(p.A, 0), 8, "init generator");
      S.check(p.D, at(p.D, s * p.ldD), 8, "init shift");
      S.check(p.R, at(p.R, i), 8, "init radius");
    }
  }
}

// ------------------------------------------------------------------ sweep
constexpr int kTrLd = 18;

// Factor reads of the sweep (the same for every sample): the diagonal
// tile's blocks by rows, and the blocks of earlier row blocks that the
// matrix cores read (lane l: entry (4 kstep + l / 16) 16 + l % 16).
void replay_sweep_factor(const SweepParams &p, bool tri, int64_t tile_doubles) {
  constexpr int SB = kSweepBlock;
  const int nb = (p.mj + SB - 1) / SB;
  const int64_t seg = tile_doubles * 8;
  int64_t blk = 0;
  for (int q = 0; q < nb; ++q) {
    if (q > 0) {
      const int64_t bq = static_cast<int64_t>(q) * (q + 1) / 2 * SB * SB;
      for (int pb = 0; pb < q; ++pb)
        for (int ks = 0; ks < 4; ++ks)
          for (int lane = 0; lane < 64; ++lane)
            S.check_seg(p.B, seg, at(p.B, bq + pb * SB * SB + ks * 64 + lane), 8, "sweep factor block");
      blk += static_cast<int64_t>(q) * SB * SB;
      // transposition in two halves: rows r = 2h, 2h + 1 of tile mt hold
      // samples 16 r + 4 (l / 16) + mt
      for (int lane = 0; lane < 64; ++lane)
        for (int h = 0; h < 2; ++h)
          for (int mt = 0; mt < 4; ++mt)
            for (int r = 2 * h; r < 2 * h + 2; ++r) {
              const int at_lds = (4 * (lane / 16 + 4 * r) + mt - 32 * h) * kTrLd + (lane & 15);
              if (at_lds < 0 || at_lds >= 32 * kTrLd) S.fail("sweep lds", 0, 8, "(index)");
            }
    }
    const int rows = std::min(SB, p.mj - q * SB);
    S.check_seg(p.B, seg, at(p.B, blk), 8, "sweep inverse diagonal");
    for (int t = 0; t < rows; ++t) {
      const int64_t col = blk + t * SB;
      for (int i = 1; i < SB; ++i)
        if (!tri || t + i < SB) S.check_seg(p.B, seg, at(p.B, col + i), 8, "sweep column");
      if (t + 1 < rows) S.check_seg(p.B, seg, at(p.B, col + SB), 8, "sweep next inverse diagonal");
    }
    blk += SB * SB;
  }
  for (int row = 0; row < p.mj; ++row) {
    S.check(p.b, at(p.b, row), 8, "sweep upper limit");
    if (p.a) S.check(p.a, at(p.a, row), 8, "sweep lower limit");
    S.check(p.A, at(p.A + p.c0, row), 8, "sweep generator");
  }
}

void replay_sweep(const SweepParams &p, Grid g, bool two_sided, bool scaled, bool prec, int64_t tile_doubles) {
  constexpr int SB = kSweepBlock;
  const int esz = prec ? 4 : 8;
  const int nb = (p.mj + SB - 1) / SB;
  const bool tri = prec && !two_sided;
  const bool has_delta = p.Delta != nullptr;
  const int64_t dls = has_delta ? p.ld : 0;
  if (two_sided != (p.a != nullptr)) S.fail("sweep", 0, 0, "(lower limits and form disagree)");
  if (first_time(p.B, p.mj, 1, 0)) replay_sweep_factor(p, tri, tile_doubles);
  // lanes: every lane of every wave, or the first wave's ends and the last
  // live wave (its live and dead lanes at both ends)
  const int64_t nthreads = static_cast<int64_t>(g.x) * 256;
  const int64_t lw = (p.count - 1) / 64 * 64;
  std::vector<int64_t> lanes = literal ? sample_threads(nthreads, p.count)
                                       : within({0, 1, 63, lw, p.count - 1, p.count, lw + 63}, nthreads);
  for (int64_t si : lanes) {
    const int lane = static_cast<int>(si & 63);
    const int64_t w0 = si - lane;
    if (w0 >= p.count) continue;
    const bool live = si < p.count;
    const int64_t sl = live ? si : p.count - 1;
    const int64_t s = (p.g0 + sl) / p.N;
    const uint64_t *Ds = p.D + s * p.ldD + p.c0;
    if (scaled) S.check(p.R, at(p.R, sl), 8, "sweep radius");
    S.check(p.logp, at(p.logp, sl), 8, "sweep logp read");
    for (int q = 0; q < nb; ++q) {
      if (q > 0)
        for (int64_t pb : span(0, q))
          for (int64_t ks : span(0, 4))
            {
              // one vector load of samples 4 (l % 16) .. 4 (l % 16) + 3
              const int64_t yi = w0 + 4 * (lane & 15) + static_cast<int64_t>(lane >> 4) * p.ld +
                                 (pb * SB + ks * 4) * p.ld;
              const uint64_t a = at_bytes(p.Y, yi * esz);
              if (a % (4 * esz) != 0) S.fail("sweep y (matrix cores)", a, 4 * esz, "(misaligned vector load)");
              S.check(p.Y, a, 4 * esz, "sweep y (matrix cores)");
            }
      const int rows = std::min(SB, p.mj - q * SB);
      for (int t = 0; t < rows; ++t) {
        const int row = q * SB + t;
        S.check(p.D, at(Ds, row), 8, "sweep shift");
        if (has_delta) S.check(p.Delta, at_bytes(p.Delta, (si + row * dls) * esz), esz, "sweep update");
        S.check(p.Y, at_bytes(p.Y, (si + static_cast<int64_t>(row) * p.ld) * esz), esz, "sweep y store");
      }
    }
    if (live) S.check(p.logp, at(p.logp, si), 8, "sweep logp store");
  }
}

// ------------------------------------------------------- BF16 low rank
// B (K x count, leading dimension ld) through one buffer resource per
// 32-deep step; A (rows padded to 64 RT, row-major with leading dimension
// KP) read straight; C stored to row map[row] (or row).
void replay_lr_mfma(const MfmaLrParams &p, Grid g, bool batch, int rt_launch, int64_t a_seg_elems,
                    int64_t b_seg_bytes, int64_t out_seg_bytes) {
  constexpr int NT = kLrNT, NS = NT / 4;
  const int RT = batch ? rt_launch : lr_mfma_rt(p.rows);
  if (RT != lr_mfma_rt(p.rows)) S.fail("lr_mfma", 0, 0, "(row tiles of the launch differ from the descriptor's)");
  const bool BD = p.Bd != nullptr;
  const int sz = BD ? 8 : 4;
  const void *Bp = BD ? static_cast<const void *>(p.Bd) : static_cast<const void *>(p.Bf);
  const int nrb = (p.rows + 64 * RT - 1) / (64 * RT);
  const int64_t nsb = (p.count + 16 * NT - 1) / (16 * NT);
  const unsigned total = batch ? static_cast<unsigned>(nsb) * static_cast<unsigned>(nrb) : g.x;
  if (!batch && static_cast<int64_t>(total) != nsb * nrb) S.fail("lr_mfma grid", total, 0, "(grid != blocks)");
  if (batch && (g.x % 8 || g.x < total)) S.fail("lr_mfma grid", g.x, 0, "(batched grid)");
  if (p.KP % 32 || p.KP < 32 || p.K > p.KP) S.fail("lr_mfma", p.KP, 0, "(KP)");
  const int nsteps = p.KP / 32;
  // the k offsets of the steps' loads, as issued: B at 0 and 32, A at 0,
  // then per step A at kk + 32 and B at kk + 64
  std::vector<int> kb = {0, 32}, ka = {0};
  {
    auto step = [&](int kk) {
      ka.push_back(kk + 32);
      kb.push_back(kk + 64);
    };
    for (int kk = 0; kk + 64 <= 32 * nsteps; kk += 64) {
      step(kk);
      step(kk + 32);
    }
    if (nsteps & 1) step(32 * (nsteps - 1));
  }
  // 32-bit lane offsets of the B loads (the same for every block and step)
  const uint32_t row_bytes = static_cast<uint32_t>(p.ld * sz);
  if (static_cast<int64_t>(row_bytes) != p.ld * sz) S.fail("lr_mfma", 0, 0, "(row bytes overflow)");
  if (first_time(nullptr, p.ld * sz, 1, 0))
    for (int w = 0; w < 4; ++w)
      for (int l = 0; l < 64; ++l) {
        const int kq = 8 * (l >> 4);
        const int64_t lo64 = (static_cast<int64_t>(kq) * p.ld + 16 * w + (l & 15)) * sz;
        const uint32_t lane_off = static_cast<uint32_t>((kq * p.ld + 16 * w + (l & 15)) * sz);
        for (int u = 0; u < NS; ++u)
          for (int e = 0; e < 8; ++e) {
            const int64_t off64 = lo64 + 64 * u * sz + static_cast<int64_t>(e) * row_bytes;
            const int off = static_cast<int>(lane_off + (64 * u) * sz + e * row_bytes);
            if (off64 != off || off64 < 0) S.fail("lr_mfma B offset", off64, 0, "(32-bit overflow)");
            // inside the step's resource (32 rows of the leading dimension)
            if (off64 >= 32 * static_cast<int64_t>(row_bytes)) S.fail("lr_mfma B offset", off64, 0, "(past 32 rows)");
          }
      }
  // A: independent of the sample block; once per row block and operand
  if (first_time(p.Ahi, p.KP, p.rows, RT))
    for (int rb = 0; rb < nrb; ++rb)
      for (int w = 0; w < 4; ++w)
        for (int l = 0; l < 64; ++l) {
          const int r0 = rb * 64 * RT + w * 16 * RT;
          const int kq = 8 * (l >> 4);
          std::vector<int> kas = literal ? ka : std::vector<int>{ka.front(), ka.back()};
          for (int kk : kas) {
            const int kc = std::min(kk, p.KP - 32);
            for (int rt = 0; rt < RT; ++rt) {
              const int64_t ro = static_cast<int64_t>(r0 + 16 * rt + (l & 15)) * p.KP + kc + kq;
              S.check_seg(p.Ahi, a_seg_elems * 2, at(p.Ahi, ro), 16, "lr_mfma A hi");
              S.check_seg(p.Alo, a_seg_elems * 2, at(p.Alo, ro), 16, "lr_mfma A lo");
            }
          }
        }
  std::vector<char> hit(total, 0);
  const std::vector<int64_t> sbs = literal ? span(0, nsb) : within({0, nsb - 1}, nsb);
  for (unsigned bid = 0; bid < g.x; ++bid) {
    if (batch && bid >= total) continue;
    const unsigned q = total / 8, rm = total % 8;
    const unsigned xcd = bid % 8, idx = bid / 8;
    const unsigned logical = xcd * q + std::min(xcd, rm) + idx;
    if (logical >= total || hit[logical]) {
      S.fail("lr_mfma remap", logical, 0, "(not a bijection)");
      continue;
    }
    hit[logical] = 1;
    const unsigned rb = logical % static_cast<unsigned>(nrb), sb = logical / static_cast<unsigned>(nrb);
    if (!std::binary_search(sbs.begin(), sbs.end(), static_cast<int64_t>(sb))) continue;
    const int64_t s0 = static_cast<int64_t>(sb) * (16 * NT);
    // B: the resource of each step spans bytes = (rows of [kk, min(kk + 32,
    // K))) x row_bytes from its base; a load at an offset at or past that
    // reads zero without an access, every other load is an access
    std::vector<int> kbs;
    for (int kk : kb)
      if (p.K - kk > 0) kbs.push_back(kk);
    if (!literal && kbs.size() > 2) kbs = {kbs.front(), kbs.back()};
    for (int kk : kbs) {
      const int64_t bytes64 = std::max<int64_t>(0, std::min(32, p.K - kk)) * static_cast<int64_t>(row_bytes);
      const int bytes = static_cast<int>(std::max(0, std::min(32, p.K - kk)) * row_bytes);
      if (bytes64 != bytes) S.fail("lr_mfma B range", bytes64, 0, "(32-bit overflow)");
      const uint64_t base = at_bytes(Bp, (static_cast<int64_t>(kk) * p.ld + s0) * sz);
      for (int w = 0; w < 4; ++w)
        for (int l = 0; l < 64; ++l) {
          // extremes: the sample columns 0 and 127 of the block, every k row
          if (!literal && !((w == 0 && (l & 15) == 0) || (w == 3 && (l & 15) == 15))) continue;
          const int kq = 8 * (l >> 4);
          const uint32_t lane_off = static_cast<uint32_t>((kq * p.ld + 16 * w + (l & 15)) * sz);
          for (int u = 0; u < NS; ++u) {
            if (!literal && u != (w == 0 ? 0 : NS - 1)) continue;
            for (int e = 0; e < 8; ++e) {
              const int off = static_cast<int>(lane_off + (64 * u) * sz + e * row_bytes);
              if (off < bytes) S.check_seg(Bp, b_seg_bytes, base + static_cast<uint64_t>(off), sz, "lr_mfma B load");
            }
          }
        }
    }
    // stores: lane l of wave w holds rows r0 + 16 rt + 4 (l / 16) + i and
    // samples s0 + 16 t + l % 16 (extremes: the block's first and last
    // stored sample of each row)
    const int64_t s_last = std::min<int64_t>(s0 + 16 * NT, p.count) - 1;
    for (int w = 0; w < 4; ++w)
      for (int l = 0; l < 64; ++l) {
        const int r0 = static_cast<int>(rb) * 64 * RT + w * 16 * RT;
        for (int rt = 0; rt < RT; ++rt)
          for (int i = 0; i < 4; ++i) {
            const int row = r0 + 16 * rt + 4 * (l >> 4) + i;
            if (row >= p.rows) continue;
            int64_t orow = row;
            if (p.map) {
              S.check(p.map, at(p.map, row), 4, "lr_mfma map");
              orow = map_value(p.map, row);
            }
            for (int t = 0; t < NT; ++t) {
              const int64_t s = s0 + 16 * t + (l & 15);
              if (!literal && s != s0 + (l & 15) && s != s_last - 15 + (l & 15)) continue;
              if (s < p.count) S.check_seg(p.Out, out_seg_bytes, at(p.Out, orow * p.ld + s), 4, "lr_mfma store");
            }
          }
      }
  }
  for (unsigned i = 0; i < total; ++i)
    if (!hit[i]) {
      S.fail("lr_mfma remap", i, 0, "(block never visited)");
      break;
    }
}

// -------------------------------------------------------- FP64 low rank
void replay_lr64(const LrParams &p, Grid g, bool batch, int64_t mat_seg_doubles, int64_t in_seg_doubles) {
  constexpr int TR = kLr64Tile, KC = 16;
  if (p.count <= 0 || p.rows <= 0) return;  // the launcher launches nothing
  const int64_t nsb = (p.count + TR - 1) / TR;
  const int nch = p.K > 0 ? (p.K + KC - 1) / KC : 0;
  const std::vector<int64_t> sbs = literal ? span(0, g.x) : within({0, nsb - 1, static_cast<int64_t>(g.x) - 1}, g.x);
  for (unsigned by = 0; by < g.y; ++by)
    for (int64_t bx : sbs) {
      if (batch && (bx * TR >= p.count || static_cast<int>(by) * TR >= p.rows)) continue;
      if (!batch && (bx >= nsb || static_cast<int>(by) * TR >= round_up(p.rows, TR))) S.fail("lr64 grid", bx, 0, "");
      const int r0 = static_cast<int>(by) * TR;
      const int64_t s0 = bx * TR;
      for (int t = 0; t < 256; ++t) {
        const int lr = t & (TR - 1), lc = t >> 7;
        const bool oka = r0 + lr < p.lda, okb = s0 + lr < p.count;
        const uint32_t ua = oka ? static_cast<uint32_t>(r0 + lr) : 0u;
        const int64_t ub = okb ? s0 + lr : 0;
        // rows k of the chunks read by this thread (row 0 stands in past K)
        std::vector<int> ks;
        for (int ch = 0; ch < nch; ++ch)
          for (int j = 0; j < KC / 2; ++j) {
            const int k = ch * KC + lc + 2 * j;
            ks.push_back(k < p.K ? k : 0);
          }
        if (!literal && ks.size() > 2) {
          const auto mm = std::minmax_element(ks.begin(), ks.end());
          ks = {*mm.first, *mm.second};
        }
        for (int kk : ks) {
          S.check_seg(p.Mat, mat_seg_doubles * 8, at(p.Mat + static_cast<int64_t>(kk) * p.lda, ua), 8, "lr64 A");
          S.check_seg(p.In, in_seg_doubles * 8, at(p.In + static_cast<int64_t>(kk) * p.ld, ub), 8, "lr64 B");
        }
        const int w = t >> 6, l = t & 63;
        const int rw = r0 + (w >> 1) * 64;
        const int64_t sw = s0 + (w & 1) * 64;
        for (int si = 0; si < 4; ++si)
          for (int r = 0; r < 4; ++r) {
            const int row = rw + si * 16 + (l >> 4) + 4 * r;
            if (row >= p.rows) continue;
            for (int sj = 0; sj < 4; ++sj) {
              const int64_t s = sw + sj * 16 + (l & 15);
              if (!literal && sj != 0 && sj != 3) continue;
              if (s < p.count) S.check(p.Out, at(p.Out, static_cast<int64_t>(row) * p.ld + s), 8, "lr64 store");
            }
          }
      }
    }
}

// ------------------------------------------------- FP64 projection (VALU)
void replay_zproj_f64(const LrParams &p, Grid g, int64_t mat_seg_doubles, int64_t in_seg_doubles) {
  const std::vector<int64_t> threads = sample_threads(static_cast<int64_t>(g.x) * 256, p.count);
  for (unsigned by = 0; by < g.y; ++by) {
    const int c0 = static_cast<int>(by) * kLrRows;
    if (c0 >= p.rows) continue;
    // the panel rows (the same for every sample)
    if (first_time(p.Mat, c0, p.K, 2))
      for (int64_t t : span(0, p.K))
        for (int64_t c : span(0, kLrRows))
          S.check_seg(p.Mat, mat_seg_doubles * 8, at(p.Mat + c0, t * p.lda + c), 8, "zproj panel");
    const int nc = std::min(kLrRows, p.rows - c0);
    for (int64_t si : threads) {
      if (si >= p.count) continue;
      for (int64_t t : span(0, p.K)) S.check_seg(p.In, in_seg_doubles * 8, at(p.In, si + t * p.ld), 8, "zproj y");
      for (int c = 0; c < nc; ++c) {
        S.check(p.map, at(p.map, c0 + c), 4, "zproj map");
        S.check(p.Out, at(p.Out, si + map_value(p.map, c0 + c) * p.ld), 8, "zproj store");
      }
    }
  }
}

// ------------------------------------------------------------------ reduce
void replay_reduce(const ReduceParams &p, Grid g, bool batch) {
  for (unsigned bx = 0; bx < g.x; ++bx) {
    if (batch && static_cast<int>(bx) >= p.M) continue;
    const int64_t s = bx;
    // thread t reads samples t, t + 256, ... of the shift
    for (int64_t i : span(0, p.N)) S.check(p.logp, at(p.logp, s * p.N + i), 8, "reduce logp");
    for (int k = 0; k < 3; ++k) S.check(p.part, at(p.part, 3 * s + k), 8, "reduce part");
  }
}

// ------------------------------------------------------------------- factors
// Planted mistakes (the replay's own check): a chunk buffer of Z short by
// a row (32 in the precision form), a row map entry one past its Z.
bool g_plant_short_z = false, g_plant_map = false;

enum Profile { kZero, kCap, kFull, kRandom };
const char *profile_name(Profile p) {
  static const char *n[] = {"zero", "cap", "full", "random"};
  return n[p];
}

uint64_t splitmix(uint64_t &x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct Factor {
  tlrqmc_factor f;
  std::vector<int32_t> zmap, zmapp;
};

// Ranks: zero, min(tile sizes, cap), the full tile size, or random in
// [0, min(tile sizes, cap)] with a quarter of the tiles at zero.
void make_factor(Factor &F, int64_t n, int m, Profile prof, int cap, uint64_t seed) {
  tlrqmc_factor &f = F.f;
  const int r = static_cast<int>((n + m - 1) / m);
  std::vector<int32_t> ranks(static_cast<size_t>(r) * r, 0);
  auto rows = [&](int i) { return static_cast<int>(std::min<int64_t>(m, n - static_cast<int64_t>(i) * m)); };
  for (int i = 1; i < r; ++i)
    for (int j = 0; j < i; ++j) {
      const int full = std::min(rows(i), rows(j));
      const int kmax = cap > 0 ? std::min(full, cap) : full;
      int k = 0;
      if (prof == kCap) k = kmax;
      else if (prof == kFull) k = full;
      else if (prof == kRandom) {
        const uint64_t u = splitmix(seed);
        k = (u % 4 == 0) ? 0 : static_cast<int>((u >> 8) % (kmax + 1));
      }
      ranks[static_cast<size_t>(i) * r + j] = k;
    }
  factor_geometry(&f, n, m, ranks.data());
  factor_layout(&f);
  F.zmap.assign(std::max<int64_t>(f.zmap_off[r], 1), 0);
  F.zmapp.assign(std::max<int64_t>(f.zmap_off[r], 1), 0);
  for (int i = 0; i < r; ++i) factor_zmaps(&f, i, F.zmap.data() + f.zmap_off[i], F.zmapp.data() + f.zmap_off[i]);
  // every map target inside Z (k_tot rows) and the padded Z (zp_tot rows),
  // each row of Z the target of exactly one column
  std::vector<char> seen(f.k_tot, 0);
  for (int64_t c = 0; c < f.zmap_off[r]; ++c) {
    if (F.zmap[c] < 0 || F.zmap[c] >= f.k_tot || seen[F.zmap[c]]++) S.fail("zmap", c, 0, "(target)");
    if (F.zmapp[c] < 0 || F.zmapp[c] >= f.zp_tot) S.fail("zmapp", c, 0, "(target outside the padded Z)");
  }
  if (f.zmap_off[r] != f.k_tot) S.fail("zmap", f.zmap_off[r], 0, "(columns != rows of Z)");
  if (g_plant_map && f.zmap_off[r] > 0) {
    F.zmap[f.zmap_off[r] - 1] = static_cast<int32_t>(f.k_tot);
    F.zmapp[f.zmap_off[r] - 1] = static_cast<int32_t>(f.zp_tot);
  }
}

void place_factor(Factor &F) {
  tlrqmc_factor &f = F.f;
  size_t sz[8];
  factor_device_sizes(&f, sz);
  S.regions.clear();
  g_done.clear();
  g_seen.clear();
  f.d_diag = static_cast<double *>(S.alloc("diagonal tiles", sz[0]));
  f.d_urow = static_cast<double *>(S.alloc("U_row", sz[1]));
  f.d_vpan = static_cast<double *>(S.alloc("V_panel", sz[2]));
  f.d_zmap = static_cast<int32_t *>(S.alloc("zmap", sz[3]));
  f.d_gen = static_cast<uint64_t *>(S.alloc("generators", sz[4]));
  f.d_ubf = static_cast<unsigned short *>(S.alloc("U_row BF16", sz[5]));
  f.d_vbf = static_cast<unsigned short *>(S.alloc("V_panel BF16", sz[6]));
  f.d_zmapp = static_cast<int32_t *>(S.alloc("padded zmap", sz[7]));
  g_maps.clear();
  if (f.d_zmap) g_maps[reinterpret_cast<uint64_t>(f.d_zmap)] = F.zmap.data();
  if (f.d_zmapp) g_maps[reinterpret_cast<uint64_t>(f.d_zmapp)] = F.zmapp.data();
}

ChunkBuffers place_chunk(const tlrqmc_factor &f, bool prec, bool scaled, int64_t ld, const std::string &tag,
                         const std::function<void *(const std::string &, int64_t)> &take) {
  int64_t lb[4];
  chunk_buffer_bytes(&f, prec, scaled, ld, lb);
  // (the padded Z of the precision form ends in up to 31 rows no kernel
  // touches: 32 rows short)
  if (g_plant_short_z && lb[2] > 0) lb[2] -= (prec ? 32 * 4 : 8) * ld;
  const char *names[4] = {"Y", "update", "Z", "radii"};
  void *b[4];
  for (int q = 0; q < 4; ++q) b[q] = lb[q] > 0 ? take(std::string(names[q]) + " " + tag, lb[q]) : nullptr;
  ChunkBuffers c;
  c.Y = b[0];
  c.R = static_cast<double *>(b[3]);
  if (prec) {
    c.DlF = static_cast<float *>(b[1]);
    c.ZF = static_cast<float *>(b[2]);
  } else {
    c.Dl = static_cast<double *>(b[1]);
    c.Z = static_cast<double *>(b[2]);
  }
  return c;
}

// ---------------------------------------------------------- one tile step
int64_t g_launches = 0;
using BatchGrid = std::function<Grid(char)>;

void replay_tile(const tlrqmc_factor &f, int j, const ChunkRun &c, bool two_sided, bool scaled,
                 const BatchGrid *batch) {
  const TileLaunch t = tile_launch(&f, j, c);
  const int64_t ld = c.ld;
  if (t.delta) {
    ++g_launches;
    if (c.prec ? !new_descriptor(t.delta_mfma) : !new_descriptor(t.delta_f64)) {
    } else if (c.prec) {
      const MfmaLrParams &p = t.delta_mfma;
      replay_lr_mfma(p, batch ? (*batch)('d') : lr_mfma_grid(p.count, p.rows), batch != nullptr, lr_mfma_rt(p.rows),
                     f.ubf_size[j], f.krow[j] * ld * 4, static_cast<int64_t>(f.tm[j]) * ld * 4);
    } else {
      const LrParams &p = t.delta_f64;
      replay_lr64(p, batch ? (*batch)('D') : lr64_grid(p.count, p.rows, 1), batch != nullptr,
                  f.urow_off[j + 1] - f.urow_off[j], f.krow[j] * ld);
    }
  }
  ++g_launches;
  replay_sweep(t.sweep, batch ? (*batch)('s') : sweep_grid(t.sweep.count), two_sided, scaled, c.prec,
               f.diag_off[j + 1] - f.diag_off[j]);
  if (t.zproj) {
    ++g_launches;
    if (c.prec ? !new_descriptor(t.zproj_mfma) : !new_descriptor(t.zproj_f64)) {
    } else if (c.prec) {
      const MfmaLrParams &p = t.zproj_mfma;
      replay_lr_mfma(p, batch ? (*batch)('z') : lr_mfma_grid(p.count, p.rows), batch != nullptr, lr_mfma_rt(p.rows),
                     f.vbf_size[j], static_cast<int64_t>(f.tm[j]) * ld * 4, f.zp_tot * ld * 4);
    } else {
      const LrParams &p = t.zproj_f64;
      replay_zproj_f64(p, batch ? (*batch)('Z') : zproj_f64_grid(p.count, p.rows), f.vpan_off[j + 1] - f.vpan_off[j],
                       static_cast<int64_t>(f.tm[j]) * ld);
    }
  }
}

// ----------------------------------------------- estimator call (one process)
struct Call {
  int64_t N;
  int M;
  bool prec;
  double nu;
  bool two_sided;
  int64_t g0 = 0, count = -1;  // default: the whole estimate, reduced
  int64_t fixed = -1;          // bytes of a no-allocation region, or -1
  int64_t chunk = 0;           // requested samples per chunk
};

// The estimator driver's sequence: per-call arrays, chunk buffers per
// worker stream, then rounds of chunks (init, tile steps) and, for a full
// estimate, the reduction.  Returns false when the call is refused for
// memory before any launch.
bool replay_call(Factor &F, const Call &k) {
  tlrqmc_factor &f = F.f;
  const int64_t n = f.n;
  const bool reduce = k.count < 0;
  const int64_t count = reduce ? k.N * k.M : k.count;
  const bool scaled = k.nu > 0;
  place_factor(F);
  const int64_t call_bytes = estimator_call_bytes(n, k.M, count, k.two_sided, reduce);
  const ChunkPlan cp = plan_chunks(&f, k.prec, count, k.chunk, k.fixed, call_bytes);
  if (cp.chunk == 0) return false;
  if (cp.chunk % 256 || cp.chunk > kMaxChunk) S.fail("chunk", cp.chunk, 0, "(size)");
  const int64_t ld = cp.chunk;
  // in a fixed region every buffer is a 256-aligned piece of it; each piece
  // is an allocation of its own here, so a write into a neighbour is caught
  int64_t used = 0;
  bool fits = true;
  auto take = [&](const std::string &name, int64_t bytes) -> void * {
    if (k.fixed >= 0) {
      const int64_t need = round_up(bytes ? bytes : 1, 256);
      if (used + need > k.fixed) {
        fits = false;
        return nullptr;
      }
      used += need;
    }
    return S.alloc(name, bytes);
  };
  double *d_a = k.two_sided ? static_cast<double *>(take("lower limits", 8 * n)) : nullptr;
  double *d_b = static_cast<double *>(take("upper limits", 8 * n));
  uint64_t *d_D = static_cast<uint64_t *>(take("shifts", 8 * static_cast<int64_t>(k.M) * (n + 1)));
  double *d_logp = static_cast<double *>(take("log P", 8 * count));
  double *d_part = reduce ? static_cast<double *>(take("partial sums", 8 * 3 * k.M)) : nullptr;
  std::vector<ChunkBuffers> lanes;
  for (int w = 0; w < cp.nstream; ++w) lanes.push_back(place_chunk(f, k.prec, scaled, ld, "lane " + std::to_string(w), take));
  if (!fits) {
    S.fail("fixed region", used, 0, "(the chunk plan does not fit the region)");
    return true;
  }
  const std::string ctx0 = S.context;
  for (int64_t base = 0; base < count; base += ld * cp.nstream)
    for (int w = 0; w < cp.nstream; ++w) {
      const int64_t c0 = base + w * ld;
      if (c0 >= count) continue;
      const ChunkRun run{k.g0 + c0, std::min(ld, count - c0), k.N, ld, k.prec, lanes[w], d_a, d_b, d_D, d_logp + c0};
      S.context = ctx0 + " chunk@" + std::to_string(c0) + " init";
      ++g_launches;
      replay_init(init_launch(&f, run, k.nu), init_grid(run.count));
      for (int j = 0; j < f.r; ++j) {
        S.context = ctx0 + " chunk@" + std::to_string(c0) + " tile " + std::to_string(j);
        replay_tile(f, j, run, k.two_sided, scaled, nullptr);
      }
    }
  if (reduce) {
    S.context = ctx0 + " reduce";
    ++g_launches;
    replay_reduce(ReduceParams{k.N, k.M, d_logp, d_part}, reduce_grid(k.M), false);
  }
  S.context = ctx0;
  return true;
}

// ------------------------------------------------------ served request slots
// A request's slots through the batched kernels.  A batched grid is taken
// as large as a step can make it (the slot cap in samples, the largest row
// count of the mix): blocks past a descriptor's own extent leave at once,
// so this replays a superset of the blocks of any real step.
void replay_served(Factor &F, int64_t N, int M, bool prec, double nu, bool two_sided, int max_rows) {
  tlrqmc_factor &f = F.f;
  const int64_t n = f.n, count = N * M;
  const bool scaled = nu > 0;
  place_factor(F);
  const SlotPlan sp = plan_slots(&f, prec, scaled, count);
  if (sp.chunk % 256 || sp.chunk > round_up(kSlotSamples, 256) || sp.nslots < 1) S.fail("slot", sp.chunk, 0, "(size)");
  double *d_b = static_cast<double *>(S.alloc("upper limits", 8 * n));
  double *d_a = two_sided ? static_cast<double *>(S.alloc("lower limits", 8 * n)) : nullptr;
  uint64_t *d_D = static_cast<uint64_t *>(S.alloc("shifts", 8 * static_cast<int64_t>(M) * (n + 1)));
  double *d_logp = static_cast<double *>(S.alloc("log P", 8 * count));
  double *d_part = static_cast<double *>(S.alloc("partial sums", 8 * 3 * M));
  const int64_t maxc = round_up(kSlotSamples, 256);
  const BatchGrid grid = [&](char kind) -> Grid {
    switch (kind) {
      case 'd':
      case 'z': return lr_mfma_batch_grid(1, std::max(lr_mfma_blocks(maxc, 64), lr_mfma_blocks(maxc, max_rows)));
      case 'D': return lr64_batch_grid(1, maxc, max_rows);
      case 'Z': return zproj_f64_batch_grid(1, maxc, max_rows);
      default: return sweep_batch_grid(1, maxc);
    }
  };
  auto take = [&](const std::string &name, int64_t bytes) { return S.alloc(name, bytes); };
  const std::string ctx0 = S.context;
  for (int sl = 0; sl < sp.nslots; ++sl) {
    const ChunkBuffers b = place_chunk(f, prec, scaled, sp.chunk, "slot " + std::to_string(sl), take);
    const int64_t c0 = static_cast<int64_t>(sl) * sp.chunk;
    const ChunkRun run{c0, std::min(sp.chunk, count - c0), N, sp.chunk, prec, b, d_a, d_b, d_D, d_logp + c0};
    S.context = ctx0 + " slot " + std::to_string(sl) + " init";
    ++g_launches;
    replay_init(init_launch(&f, run, nu), init_batch_grid(1, maxc));
    for (int j = 0; j < f.r; ++j) {
      S.context = ctx0 + " slot " + std::to_string(sl) + " tile " + std::to_string(j);
      replay_tile(f, j, run, two_sided, scaled, &grid);
    }
  }
  S.context = ctx0 + " reduce";
  ++g_launches;
  replay_reduce(ReduceParams{N, M, d_logp, d_part}, reduce_batch_grid(1, 64), true);
  S.context = ctx0;
}

// Descriptors of one serving step fit its staging buffer: a slot adds at
// most one descriptor of each kind, and each of the groups starts on 256.
void check_step_staging() {
  constexpr int kMaxSlots = 64, kGroups = 1 + 4 + 2 + 8 + 1;
  const size_t per_slot = sizeof(InitParams) + 2 * sizeof(MfmaLrParams) + 2 * sizeof(LrParams) + sizeof(SweepParams) +
                          sizeof(ReduceParams);
  if (kMaxSlots * per_slot + kGroups * 256 > 256 * 1024) S.fail("step staging", 0, 0, "(descriptors)");
}

// ----------------------------------------------------------------- cases
struct Case {
  std::string name;
  bool literal;
  std::function<void()> run;
};

std::vector<Case> cases() {
  std::vector<Case> v;
  auto est = [&](const std::string &name, bool lit, int64_t n, int m, Profile prof, int cap, Call k) {
    v.push_back({name, lit, [=]() {
                   Factor F;
                   make_factor(F, n, m, prof, cap, 0x5EED + static_cast<uint64_t>(n) * 31 + m);
                   if (!replay_call(F, k)) {
                     if (k.fixed < 0) S.fail("call", 0, 0, "(refused without a fixed region)");
                     else std::printf("  %s: refused (does not fit the fixed region)\n", S.context.c_str());
                   }
                 }});
  };
  auto srv = [&](const std::string &name, int64_t n, Profile prof, int cap, bool prec, double nu, bool two_sided,
                 int64_t N = 10000) {
    v.push_back({name, false, [=]() {
                   Factor F;
                   make_factor(F, n, 128, prof, cap, 0xC0FFEE + static_cast<uint64_t>(n));
                   replay_served(F, N, 10, prec, nu, two_sided, 128 * 127);
                 }});
  };
  // the benchmark workloads at full size: n = 256 (one tile), 4,096 (m 64,
  // cap 32), 16,384 (m 256, nu 7), 65,536 (m 512, cap 64); N x 10 shifts
  for (int prec = 0; prec < 2; ++prec) {
    const std::string f = prec ? "prec" : "fp64";
    est("cfg1-dense-" + f, true, 256, 256, kZero, 0, Call{10000, 10, prec == 1, 0.0, false});
    for (Profile p : {kCap, kRandom, kZero, kFull})
      est("cfg2-" + f + "-" + profile_name(p), false, 4096, 64, p, 32, Call{20000, 10, prec == 1, 0.0, false});
    for (Profile p : {kCap, kRandom})
      est("cfg3-" + f + "-" + profile_name(p), false, 16384, 256, p, 64, Call{40000, 10, prec == 1, 7.0, false});
    for (Profile p : {kCap, kRandom})
      est("cfg4-" + f + "-" + profile_name(p), false, 65536, 512, p, 64, Call{20000, 10, prec == 1, 0.0, false});
  }
  est("cfg3-prec-full", false, 16384, 256, kFull, 0, Call{40000, 10, true, 7.0, false});
  // the serving stream's requests: n = 32^2 .. 128^2, tiles of 128, MVN and MVT
  for (int64_t n : {1024, 4096, 9216, 16384})
    for (int prec = 0; prec < 2; ++prec)
      srv("serve-n" + std::to_string(n) + (prec ? "-prec" : "-fp64"), n, kRandom, 64, prec == 1,
          n == 4096 ? 5.0 : 0.0, false);
  // full ranks: slots of a few hundred samples (fewer samples replayed)
  srv("serve-n9216-full-mvt-prec", 9216, kFull, 0, true, 10.0, false, 600);
  srv("serve-n16384-full-mvt-prec", 16384, kFull, 0, true, 10.0, false, 300);
  srv("serve-n1024-full-two-sided-prec", 1024, kFull, 0, true, 0.0, true);
  srv("serve-n1024-full-two-sided-fp64", 1024, kFull, 0, false, 5.0, true);
  // every form, ragged tiles, tiny and odd sample counts, thread by thread
  int id = 0;
  for (int64_t n : {1, 2, 15, 17, 100, 333, 1000})
    for (int m : {16, 32, 64, 100, 128})
      for (int prec = 0; prec < 2; ++prec)
        for (int form = 0; form < 4; ++form)
          for (int64_t N : {1, 37, 300}) {
            const bool two = form & 1;
            const double nu = (form & 2) ? 5.0 : 0.0;
            const Profile p = static_cast<Profile>(id % 4);
            const int M = 2 + id % 3;
            ++id;
            est("small-n" + std::to_string(n) + "-m" + std::to_string(m) + (prec ? "-prec" : "-fp64") +
                    (two ? "-two" : "-one") + (nu > 0 ? "-mvt" : "-mvn") + "-N" + std::to_string(N) + "-" +
                    profile_name(p),
                true, n, m, p, 0, Call{N, M, prec == 1, nu, two});
          }
  // chunks of a requested size; slices of the sample range (no
  // reduction); two worker streams; the no-allocation region
  est("small-chunked-prec", true, 1000, 64, kFull, 0, Call{5000, 4, true, 5.0, true, 0, -1, -1, 700});
  est("small-chunked-fp64", true, 1000, 100, kRandom, 0, Call{5000, 4, false, 0.0, false, 0, -1, -1, 1300});
  est("small-slice-prec", true, 900, 64, kRandom, 0, Call{3000, 5, true, 0.0, false, 4321, 2500});
  est("small-slice-fp64", true, 900, 128, kCap, 24, Call{3000, 5, false, 7.0, true, 1, 7000});
  est("streams-fp64", false, 300, 64, kFull, 0, Call{70000, 2, false, 0.0, false});
  est("streams-prec", false, 300, 64, kFull, 0, Call{70000, 2, true, 3.0, true});
  for (int prec = 0; prec < 2; ++prec) {
    const std::string f = prec ? "prec" : "fp64";
    const int64_t region = int64_t{256} << 20;
    // the full-size factors, fewer samples (the region holds chunks of 256
    // to 512 samples of them)
    est("noalloc-cfg2-" + f, false, 4096, 64, kCap, 32, Call{1000, 4, prec == 1, 0.0, false, 0, -1, region});
    est("noalloc-cfg3-" + f, false, 16384, 256, kCap, 64, Call{400, 4, prec == 1, 7.0, false, 0, -1, region});
    est("noalloc-1500-" + f, false, 1500, 128, kRandom, 0, Call{40000, 8, prec == 1, 7.0, true, 0, -1, region});
    est("small-noalloc-chunk-" + f, true, 700, 64, kFull, 0, Call{3000, 6, prec == 1, 0.0, true, 0, -1, region, 300});
  }
  // planted mistakes: each must be reported (run only when named)
  for (int prec = 0; prec < 2; ++prec) {
    const std::string f = prec ? "prec" : "fp64";
    v.push_back({"plant-short-z-" + f, true, [=]() {
                   g_plant_short_z = true;
                   Factor F;
                   make_factor(F, 300, 64, kFull, 0, 7);
                   replay_call(F, Call{100, 3, prec == 1, 0.0, false});
                   g_plant_short_z = false;
                 }});
    v.push_back({"plant-map-" + f, true, [=]() {
                   g_plant_map = true;
                   Factor F;
                   make_factor(F, 300, 64, kRandom, 0, 7);
                   g_plant_map = false;
                   replay_call(F, Call{100, 3, prec == 1, 0.0, false});
                 }});
  }
  return v;
}

}  // namespace

int main(int argc, char **argv) {
  check_step_staging();
  const std::vector<Case> all = cases();
  std::vector<std::string> want(argv + 1, argv + argc);
  int ran = 0, quiet = 0;
  int planted = 0, caught = 0;
  for (const Case &c : all) {
    const bool plant = c.name.rfind("plant-", 0) == 0;
    bool pick = want.empty() && !plant;
    for (const std::string &w : want) pick = pick || c.name.rfind(w, 0) == 0;
    if (!pick) continue;
    literal = c.literal;
    S.context = c.name;
    const uint64_t c0 = S.checks;
    const int64_t f0 = S.failures, l0 = g_launches;
    c.run();
    if (plant) {
      // a planted mistake must be reported; it does not count as a failure
      ++planted;
      caught += S.failures > f0;
      std::printf("%-36s %s\n", c.name.c_str(), S.failures > f0 ? "caught" : "MISSED");
      S.failures = f0;
      continue;
    }
    ++ran;
    if (c.name.rfind("small-n", 0) == 0 && S.failures == f0) {
      ++quiet;
      continue;
    }
    std::printf("%-36s %-8s %8" PRId64 " launches %13" PRIu64 " accesses  %s\n", c.name.c_str(),
                c.literal ? "literal" : "extremes", g_launches - l0, S.checks - c0, S.failures == f0 ? "ok" : "FAILED");
    std::fflush(stdout);
  }
  std::printf("cases %d (%d small ones not listed), launches %" PRId64 ", accesses checked %" PRIu64
              ", outside their allocation %" PRId64 "\n",
              ran, quiet, g_launches, S.checks, S.failures);
  if (planted) std::printf("planted mistakes %d, caught %d\n", planted, caught);
  return S.failures == 0 && (ran > 0 || planted > 0) && caught == planted ? 0 : 1;
}

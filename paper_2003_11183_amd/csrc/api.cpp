// C ABI of libtlrqmc: context, factor objects and the estimator driver.
//
// The estimator (Section 2.1 and Section 3.4 of the paper) runs, for each
// chunk of samples, one pass over the r diagonal tiles: the low-rank limit
// update of tile j, the SOV sweep of its rows and the rank-space projection
// of its y values, then one reduction per shift.  Student-t problems
// (Section 2.2, Eq. 4) add a per-sample chi radius computed at chunk start.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <memory>
#include <string>
#include <vector>

#include "internal.hpp"

namespace tlrqmc {

namespace {
thread_local std::string g_error;
}

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

void clear_error() { g_error.clear(); }

// Estimate from per-shift partial sums (max, sum exp(lp - max), dead
// count): Section 2.1 (mean over shifts of the sample means) and Section 4
// (standard error over the shift means, relative error).
void estimate_from_parts(const std::vector<double> &part, int M, int64_t N, tlrqmc_result *out) {
  std::vector<double> Ls(M);
  double mx = -INFINITY;
  int64_t dead = 0;
  for (int s = 0; s < M; ++s) {
    const double pm = part[3 * s], ps = part[3 * s + 1];
    Ls[s] = (pm > -INFINITY && ps > 0.0) ? pm + std::log(ps) - std::log(static_cast<double>(N)) : -INFINITY;
    mx = std::max(mx, Ls[s]);
    dead += static_cast<int64_t>(part[3 * s + 2]);
  }
  out->n_dead = dead;
  out->n_shifts = M;
  for (int s = 0; s < 64; ++s) out->log_p_shift[s] = s < M ? Ls[s] : 0.0;
  if (!(mx > -INFINITY)) {
    out->log_p = -INFINITY;
    out->p = 0.0;
    out->std_err = 0.0;
    out->rel_err = std::numeric_limits<double>::quiet_NaN();
    return;
  }
  double mean = 0.0;
  for (int s = 0; s < M; ++s) mean += std::exp(Ls[s] - mx);
  mean /= M;
  double ss = 0.0;
  for (int s = 0; s < M; ++s) {
    const double d = std::exp(Ls[s] - mx) - mean;
    ss += d * d;
  }
  const double se = std::sqrt(ss / (static_cast<double>(M) * (M - 1)));
  out->log_p = mx + std::log(mean);
  out->p = std::exp(out->log_p);
  out->std_err = se * std::exp(mx);
  out->rel_err = se / mean;
}

namespace {


// Start and stop events of every launch (marked by the launch itself),
// summed per kernel kind.  The events come from the context's pool and go
// back to it.
struct Profiler {
  bool on;
  tlrqmc_ctx *ctx;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> marks;
  Profiler(bool enable, tlrqmc_ctx *c) : on(enable), ctx(c) {}
  ~Profiler() {
    for (auto &m : marks) {
      ctx->event_pool.push_back(m.second.first);
      ctx->event_pool.push_back(m.second.second);
    }
  }
  hipEvent_t take() {
    hipEvent_t e = nullptr;
    if (!ctx->event_pool.empty()) {
      e = ctx->event_pool.back();
      ctx->event_pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
    }
    return e;
  }
  // the events of the next launch of this kind (none when profiling is off)
  LaunchEvents next(int kind) {
    LaunchEvents ev;
    if (!on) return ev;
    ev.start = take();
    ev.stop = ev.start ? take() : nullptr;
    if (!ev.stop) {
      if (ev.start) ctx->event_pool.push_back(ev.start);
      return LaunchEvents{};
    }
    marks.push_back({kind, {ev.start, ev.stop}});
    return ev;
  }
  // Sum of launch durations and, per kind, the union of the launch
  // intervals (launches on different streams may overlap), both measured
  // from the reference event ref.
  void collect(tlrqmc_result *r, hipEvent_t ref) {
    std::vector<std::vector<std::pair<float, float>>> iv(TLRQMC_KERNEL_KINDS);
    for (int k = 0; k < TLRQMC_KERNEL_KINDS; ++k) {
      r->kernel_seconds[k] = 0.0;
      r->kernel_busy_seconds[k] = 0.0;
      r->kernel_launches[k] = 0;
    }
    for (auto &m : marks) {
      float t0 = 0.f, t1 = 0.f;
      (void)hipEventElapsedTime(&t0, ref, m.second.first);
      (void)hipEventElapsedTime(&t1, ref, m.second.second);
      r->kernel_seconds[m.first] += (t1 - t0) * 1e-3;
      r->kernel_launches[m.first] += 1;
      iv[m.first].push_back({t0, t1});
    }
    for (int k = 0; k < TLRQMC_KERNEL_KINDS; ++k) {
      auto &v = iv[k];
      std::sort(v.begin(), v.end());
      double busy = 0.0, cs = -1.0, ce = -1.0;
      for (auto &x : v) {
        if (x.first > ce) {
          if (ce > cs) busy += ce - cs;
          cs = x.first;
          ce = x.second;
        } else if (x.second > ce) {
          ce = x.second;
        }
      }
      if (ce > cs) busy += ce - cs;
      r->kernel_busy_seconds[k] = busy * 1e-3;
    }
  }
};

bool check_launch(const char *what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    fail(TLRQMC_EDEVICE, "launch of %s failed: %s", what, hipGetErrorString(e));
    return false;
  }
  return true;
}

// After a failed launch or copy: drain the streams, keep the first message.
int fail_device(tlrqmc_ctx *ctx, size_t nworkers) {
  const hipError_t e = hipGetLastError();
  (void)hipStreamSynchronize(ctx->stream);
  for (size_t w = 0; w < nworkers && w < ctx->workers.size(); ++w) (void)hipStreamSynchronize(ctx->workers[w]);
  if (tlrqmc_last_error()[0] == '\0') fail(TLRQMC_EDEVICE, "HIP error: %s", hipGetErrorString(e));
  return TLRQMC_EDEVICE;
}

// A fixed device region handed out by a bump pointer (256-byte aligned
// pieces); take() returns null once it is used up.
struct FixedRegion {
  char *p;
  size_t left;
  void *take(size_t bytes) {
    const size_t need = static_cast<size_t>(round_up(static_cast<int64_t>(bytes ? bytes : 1), 256));
    if (need > left) return nullptr;
    void *q = p;
    p += need;
    left -= need;
    return q;
  }
};

// Shared driver of mvn_prob, mvt_prob, tlrqmc_sample_logp and
// tlrqmc_prob_noalloc.  Samples g0 .. g0+count-1 of the flattened (shift,
// k) index space are swept; a full estimate (reduce = true) needs g0 = 0 and
// count = N M.  With fixed != null every device buffer comes from that
// region instead of the allocator, the chunks are sized to fit it, and the
// call runs on the context stream alone with no events (so it creates
// nothing on the device); its seconds are host wall time.
int run_estimator(tlrqmc_ctx *ctx, const tlrqmc_factor *f, const double *a, const double *b,
                  double nu, const tlrqmc_qmc_opts *opts, int64_t g0, int64_t count,
                  bool reduce, double *logp_host, tlrqmc_result *out, FixedRegion *fixed = nullptr) {
  clear_error();
  if (!ctx || !f || !a || !b || !opts) return fail(TLRQMC_EINVAL, "null argument");
  if (f->ctx != ctx) return fail(TLRQMC_EINVAL, "factor belongs to another context");
  const int64_t N = opts->n_samples;
  const int M = opts->n_shifts;
  if (N < 1) return fail(TLRQMC_EINVAL, "n_samples must be >= 1");
  if (M < 2 || M > 64) return fail(TLRQMC_EINVAL, "n_shifts must be in [2, 64]");
  if (opts->precision != 0 && opts->precision != 1) return fail(TLRQMC_EINVAL, "precision must be 0 or 1");
  if (!(nu >= 0.0) || std::isinf(nu)) return fail(TLRQMC_EINVAL, "nu must be finite and > 0 (0 selects MVN)");
  if (N > (int64_t{1} << 40) / M) return fail(TLRQMC_EINVAL, "too many samples");
  const int64_t n = f->n;
  const int r = f->r;
  // limits in integration order
  std::vector<double> ap(n), bp(n);
  bool two_sided = false, empty = false;
  for (int64_t i = 0; i < n; ++i) {
    const double av = a[f->perm[i]], bv = b[f->perm[i]];
    if (std::isnan(av) || std::isnan(bv)) return fail(TLRQMC_EINVAL, "NaN limit at variable %d", f->perm[i]);
    if (av >= bv) empty = true;
    if (av > -INFINITY) two_sided = true;
    ap[i] = av;
    bp[i] = bv;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(TLRQMC_EDEVICE, "hipSetDevice failed");
  if (out) std::memset(out, 0, sizeof *out);
  if (empty) {
    if (logp_host)
      for (int64_t i = 0; i < count; ++i) logp_host[i] = -INFINITY;
    if (out) {
      std::vector<double> part(3 * M, 0.0);
      for (int s = 0; s < M; ++s) {
        part[3 * s] = -INFINITY;
        part[3 * s + 2] = static_cast<double>(N);
      }
      estimate_from_parts(part, M, N, out);
    }
    return TLRQMC_OK;
  }
  // Chunking: each sample needs Z (k_tot rows), Y and Delta (padded tile
  // rows).  Large runs are split over two worker streams so that their
  // launches overlap (see tlrqmc_ctx::workers).
  const bool prec = opts->precision == 1;
  const int64_t call_bytes = estimator_call_bytes(n, M, count, two_sided, reduce);
  const ChunkPlan cp = plan_chunks(f, prec, count, opts->chunk_samples, fixed ? static_cast<int64_t>(fixed->left) : -1,
                                   call_bytes);
  if (cp.chunk == 0)
    return fail(TLRQMC_ENOMEM,
                "the problem does not fit the %lld MiB no-allocation scratch (n = %lld, %lld samples: %lld bytes "
                "of per-call arrays plus %lld per sample, chunks of at least 256 samples)",
                static_cast<long long>(noalloc_scratch_bytes() >> 20), static_cast<long long>(n),
                static_cast<long long>(count), static_cast<long long>(call_bytes),
                static_cast<long long>(chunk_bytes_per_sample(f, prec)));
  const int nstream = cp.nstream;
  const int64_t chunk = cp.chunk;
  const int64_t ld = chunk;
  SharedDevice dev;  // no library factorization runs beside these kernels
  Scratch sc(ctx);
  auto take = [&](size_t bytes) -> void * { return fixed ? fixed->take(bytes) : sc.get<char>(bytes); };
  double *d_a = two_sided ? static_cast<double *>(take(8 * n)) : nullptr;
  double *d_b = static_cast<double *>(take(8 * n));
  uint64_t *d_D = static_cast<uint64_t *>(take(8 * static_cast<size_t>(M) * (n + 1)));
  double *d_logp = static_cast<double *>(take(8 * count));
  double *d_part = reduce ? static_cast<double *>(take(8 * 3 * M)) : nullptr;
  if (!d_b || !d_D || !d_logp || (two_sided && !d_a) || (reduce && !d_part))
    return fail(TLRQMC_ENOMEM, "device allocation failed");
  struct Lane {
    hipStream_t s;
    ChunkBuffers b;
  };
  std::vector<Lane> lanes(nstream);
  if (nstream > 1 && ctx->worker_streams(nstream) != TLRQMC_OK) return TLRQMC_EDEVICE;
  int64_t lane_bytes[4];
  chunk_buffer_bytes(f, prec, nu > 0, ld, lane_bytes);
  for (int w = 0; w < nstream; ++w) {
    Lane &L = lanes[w];
    L.s = nstream > 1 ? ctx->workers[w] : ctx->stream;
    void *got[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int k = 0; k < 4; ++k)
      if (lane_bytes[k] > 0 && !(got[k] = take(static_cast<size_t>(lane_bytes[k]))))
        return fail(TLRQMC_ENOMEM, "device allocation failed (chunk of %lld samples)", static_cast<long long>(chunk));
    L.b.Y = got[0];
    L.b.R = static_cast<double *>(got[3]);
    if (prec) {
      L.b.DlF = static_cast<float *>(got[1]);
      L.b.ZF = static_cast<float *>(got[2]);
    } else {
      L.b.Dl = static_cast<double *>(got[1]);
      L.b.Z = static_cast<double *>(got[2]);
    }
  }
  const std::vector<uint64_t> shifts = splitmix64_table(opts->seed, static_cast<int64_t>(M) * (n + 1));
  hipStream_t st = ctx->stream;
  if (two_sided && hipMemcpyAsync(d_a, ap.data(), n * 8, hipMemcpyHostToDevice, st) != hipSuccess)
    return fail(TLRQMC_EDEVICE, "copy of limits failed");
  if (hipMemcpyAsync(d_b, bp.data(), n * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(d_D, shifts.data(), shifts.size() * 8, hipMemcpyHostToDevice, st) != hipSuccess)
    return fail(TLRQMC_EDEVICE, "copy of limits or shifts failed");
  Events evs;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev_in = nullptr;
  if (!fixed) {
    ev0 = evs.make();
    ev1 = evs.make();
    ev_in = evs.make();
    if (!ev0 || !ev1 || !ev_in) return fail(TLRQMC_EDEVICE, "hipEventCreate failed");
  }
  const auto t_host0 = std::chrono::steady_clock::now();
  Profiler prof(!fixed && opts->profile != 0, ctx);
  if (ev0) (void)hipEventRecord(ev0, st);
  if (ev_in) (void)hipEventRecord(ev_in, st);
  if (nstream > 1)
    for (auto &L : lanes) (void)hipStreamWaitEvent(L.s, ev_in, 0);
  int chunks = 0;
  for (int64_t base = 0; base < count; base += chunk * nstream) {
    // one round: up to nstream chunks, enqueued tile by tile across streams
    std::vector<std::pair<int64_t, int64_t>> cs;
    for (int w = 0; w < nstream; ++w) {
      const int64_t c0 = base + w * chunk;
      if (c0 < count) cs.push_back({c0, std::min(chunk, count - c0)});
    }
    chunks += static_cast<int>(cs.size());
    std::vector<ChunkRun> runs;
    for (size_t w = 0; w < cs.size(); ++w)
      runs.push_back(ChunkRun{g0 + cs[w].first, cs[w].second, N, ld, prec, lanes[w].b, d_a, d_b, d_D,
                              d_logp + cs[w].first});
    for (size_t w = 0; w < cs.size(); ++w) {
      const Lane &L = lanes[w];
      launch_init(L.s, init_launch(f, runs[w], nu), prof.next(TLRQMC_KERNEL_INIT));
      if (!check_launch("init")) return fail_device(ctx, lanes.size());
    }
    for (int j = 0; j < r; ++j) {
      for (size_t w = 0; w < cs.size(); ++w) {
        const Lane &L = lanes[w];
        const TileLaunch t = tile_launch(f, j, runs[w]);
        if (t.delta) {
          if (prec) launch_lr_mfma(L.s, t.delta_mfma, prof.next(TLRQMC_KERNEL_DELTA));
          else launch_delta_f64(L.s, t.delta_f64, prof.next(TLRQMC_KERNEL_DELTA));
          if (!check_launch("delta")) return fail_device(ctx, lanes.size());
        }
        launch_sweep(L.s, t.sweep, two_sided, nu > 0, prec, prof.next(TLRQMC_KERNEL_SWEEP));
        if (!check_launch("sweep")) return fail_device(ctx, lanes.size());
        if (t.zproj) {
          if (prec) launch_lr_mfma(L.s, t.zproj_mfma, prof.next(TLRQMC_KERNEL_ZPROJ));
          else launch_zproj_f64(L.s, t.zproj_f64, prof.next(TLRQMC_KERNEL_ZPROJ));
          if (!check_launch("zproj")) return fail_device(ctx, lanes.size());
        }
      }
    }
  }
  // the context stream waits for the workers (the host does, if the event
  // cannot be made): every later free happens after its kernels ended
  if (nstream > 1)
    for (auto &L : lanes) {
      hipEvent_t e = evs.make();
      if (!e || hipEventRecord(e, L.s) != hipSuccess || hipStreamWaitEvent(st, e, 0) != hipSuccess)
        if (hipStreamSynchronize(L.s) != hipSuccess) return fail_device(ctx, lanes.size());
    }
  if (reduce) {
    ReduceParams rp{N, M, d_logp, d_part};
    launch_reduce(st, rp, M, prof.next(TLRQMC_KERNEL_REDUCE));
    if (!check_launch("reduce")) return fail_device(ctx, lanes.size());
  }
  if (ev1) (void)hipEventRecord(ev1, st);
  {
    std::vector<double> part(reduce ? 3 * M : 0);
    if (reduce && hipMemcpyAsync(part.data(), d_part, part.size() * 8, hipMemcpyDeviceToHost, st) != hipSuccess)
      return fail_device(ctx, lanes.size());
    if (logp_host && hipMemcpyAsync(logp_host, d_logp, count * 8, hipMemcpyDeviceToHost, st) != hipSuccess)
      return fail_device(ctx, lanes.size());
    if (hipStreamSynchronize(st) != hipSuccess) return fail_device(ctx, lanes.size());
    float ms = 0.f;
    if (ev0) (void)hipEventElapsedTime(&ms, ev0, ev1);
    else ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t_host0).count();
    if (out) {
      if (reduce) estimate_from_parts(part, M, N, out);
      out->seconds = ms * 1e-3;
      out->chunks = chunks;
      if (ev0) prof.collect(out, ev0);
    }
  }
  return TLRQMC_OK;
}

}  // namespace
}  // namespace tlrqmc

using namespace tlrqmc;

void *tlrqmc_ctx::dmalloc(size_t bytes) {
  if (has_alloc) return alloc.alloc(bytes, alloc.user);
  void *p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  return p;
}

int tlrqmc_ctx::worker_streams(int count) {
  while (static_cast<int>(workers.size()) < count) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
      return fail(TLRQMC_EDEVICE, "hipStreamCreateWithFlags failed");
    workers.push_back(s);
  }
  return TLRQMC_OK;
}

double *tlrqmc_ctx::pinned(int slot, size_t bytes) {
  if (static_cast<int>(staging.size()) <= slot) staging.resize(slot + 1, {nullptr, 0});
  auto &b = staging[slot];
  if (b.second < bytes) {
    if (b.first) (void)hipHostFree(b.first);
    b = {nullptr, 0};
    void *p = nullptr;
    const size_t want = bytes + bytes / 4;  // headroom against regrowth
    if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) return nullptr;
    b = {p, want};
  }
  return static_cast<double *>(b.first);
}

void tlrqmc_ctx::release_pinned() {
  for (auto &b : staging)
    if (b.first) (void)hipHostFree(b.first);
  staging.clear();
}

void tlrqmc_ctx::dfree(void *p) {
  if (!p) return;
  if (has_alloc) alloc.free(p, alloc.user);
  else (void)hipFree(p);
}

extern "C" {

const char *tlrqmc_last_error(void) { return g_error.c_str(); }

int tlrqmc_ctx_create(int device, void *hip_stream, const tlrqmc_allocator *alloc, tlrqmc_ctx **out) {
  clear_error();
  if (!out) return fail(TLRQMC_EINVAL, "null output pointer");
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1)
    return fail(TLRQMC_EDEVICE, "no HIP device available");
  if (device < 0 || device >= count) return fail(TLRQMC_EINVAL, "device %d out of range", device);
  if (hipSetDevice(device) != hipSuccess) return fail(TLRQMC_EDEVICE, "hipSetDevice(%d) failed", device);
  // the no-allocation entry point's scratch array: its address on this
  // device, resolved once per device with the device current
  if (noalloc_resolve(device) != TLRQMC_OK) return TLRQMC_EDEVICE;
  auto c = new tlrqmc_ctx();
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (alloc && alloc->alloc && alloc->free) {
    c->alloc = *alloc;
    c->has_alloc = true;
  }
  *out = c;
  return TLRQMC_OK;
}

void tlrqmc_ctx_destroy(tlrqmc_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  for (hipStream_t s : ctx->workers) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  }
  ctx->release_pinned();
  release_blas(ctx);
  for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
  delete ctx;
}

int tlrqmc_factor_import(tlrqmc_ctx *ctx, int64_t n, int m, const int32_t *perm, const double *diag,
                         const int32_t *ranks, const double *U, const double *V, tlrqmc_factor **out) {
  clear_error();
  if (ctx && hipSetDevice(ctx->device) != hipSuccess) return fail(TLRQMC_EDEVICE, "hipSetDevice failed");
  return factor_build(ctx, n, m, perm, diag, ranks, U, V, 0, out);
}

int tlrqmc_factor_stats(const tlrqmc_factor *f, tlrqmc_factor_info *o) {
  clear_error();
  if (!f || !o) return fail(TLRQMC_EINVAL, "null argument");
  o->n = f->n;
  o->m = f->m;
  o->r = f->r;
  o->k_tot = f->k_tot;
  o->k_max = f->k_max;
  o->cap_hits = f->cap_hits;
  o->diag_doubles = static_cast<int64_t>(f->h_diag.size());
  o->uv_doubles = static_cast<int64_t>(f->h_U.size());
  o->device_bytes = f->device_bytes;
  for (int k = 0; k < 4; ++k) o->setup_seconds[k] = f->setup_seconds[k];
  o->checksum = f->checksum;
  o->host_tiles = f->host_tiles;
  return TLRQMC_OK;
}

int tlrqmc_factor_export(const tlrqmc_factor *f, int32_t *perm, double *diag, int32_t *ranks, double *U,
                         double *V) {
  clear_error();
  if (!f) return fail(TLRQMC_EINVAL, "null factor");
  if (perm) std::memcpy(perm, f->perm.data(), f->perm.size() * 4);
  if (diag) std::memcpy(diag, f->h_diag.data(), f->h_diag.size() * 8);
  if (ranks) std::memcpy(ranks, f->rank.data(), f->rank.size() * 4);
  if (U && !f->h_U.empty()) std::memcpy(U, f->h_U.data(), f->h_U.size() * 8);
  if (V && !f->h_V.empty()) std::memcpy(V, f->h_V.data(), f->h_V.size() * 8);
  return TLRQMC_OK;
}

void tlrqmc_factor_free(tlrqmc_factor *f) {
  if (!f) return;
  if (f->ctx) {
    (void)hipSetDevice(f->ctx->device);
    (void)hipStreamSynchronize(f->ctx->stream);
    f->ctx->dfree(f->d_diag);
    f->ctx->dfree(f->d_urow);
    f->ctx->dfree(f->d_vpan);
    f->ctx->dfree(f->d_zmap);
    f->ctx->dfree(f->d_gen);
    f->ctx->dfree(f->d_ubf);
    f->ctx->dfree(f->d_vbf);
    f->ctx->dfree(f->d_zmapp);
  }
  delete f;
}

int mvn_prob(tlrqmc_ctx *ctx, const tlrqmc_factor *f, const double *a, const double *b,
             const tlrqmc_qmc_opts *opts, tlrqmc_result *out) {
  if (!opts || !out) return fail(TLRQMC_EINVAL, "null opts or result");
  return run_estimator(ctx, f, a, b, 0.0, opts, 0, opts->n_samples * opts->n_shifts, true,
                       opts->logp_out, out);
}

int mvt_prob(tlrqmc_ctx *ctx, const tlrqmc_factor *f, const double *a, const double *b, double nu,
             const tlrqmc_qmc_opts *opts, tlrqmc_result *out) {
  if (!opts || !out) return fail(TLRQMC_EINVAL, "null opts or result");
  if (!(nu > 0.0)) return fail(TLRQMC_EINVAL, "nu must be > 0");
  return run_estimator(ctx, f, a, b, nu, opts, 0, opts->n_samples * opts->n_shifts, true,
                       opts->logp_out, out);
}

int tlrqmc_prob_noalloc(tlrqmc_ctx *ctx, const tlrqmc_factor *f, const double *a, const double *b, double nu,
                        const tlrqmc_qmc_opts *opts, tlrqmc_result *out) {
  if (!opts || !out) return fail(TLRQMC_EINVAL, "null opts or result");
  if (!ctx) return fail(TLRQMC_EINVAL, "null context");
  if (!(nu >= 0.0)) return fail(TLRQMC_EINVAL, "nu must be >= 0 (0 selects MVN)");
  void *base = noalloc_scratch(ctx->device);
  if (!base) return fail(TLRQMC_EDEVICE, "no-allocation scratch not resolved on device %d", ctx->device);
  FixedRegion region{static_cast<char *>(base), static_cast<size_t>(noalloc_scratch_bytes())};
  return run_estimator(ctx, f, a, b, nu, opts, 0, opts->n_samples * opts->n_shifts, true, opts->logp_out, out,
                       &region);
}

int tlrqmc_sample_logp(tlrqmc_ctx *ctx, const tlrqmc_factor *f, const double *a, const double *b,
                       double nu, const tlrqmc_qmc_opts *opts, int32_t shift, int64_t k0,
                       int64_t count, double *logp_out) {
  if (!opts || !logp_out) return fail(TLRQMC_EINVAL, "null opts or output");
  if (shift < 0 || shift >= opts->n_shifts) return fail(TLRQMC_EINVAL, "shift out of range");
  if (count < 1 || k0 < 1 || k0 + count - 1 > opts->n_samples)
    return fail(TLRQMC_EINVAL, "samples k0..k0+count-1 must lie in 1..n_samples");
  tlrqmc_result tmp;
  return run_estimator(ctx, f, a, b, nu, opts, static_cast<int64_t>(shift) * opts->n_samples + k0 - 1,
                       count, false, logp_out, &tmp);
}

}  // extern "C"

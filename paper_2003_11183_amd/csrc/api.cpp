// C ABI of libtlrqmc: context, factor objects and the estimator driver.
//
// The estimator (Section 2.1 and Section 3.4 of the paper) runs, for each
// chunk of samples, one pass over the r diagonal tiles: the low-rank limit
// update of tile j, the SOV sweep of its rows and the rank-space projection
// of its y values, then one reduction per shift.  Student-t problems
// (Section 2.2, Eq. 4) add a per-sample chi radius computed at chunk start.
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

namespace {

// Device buffers of one estimator call, released on scope exit.
struct Scratch {
  tlrqmc_ctx *ctx;
  std::vector<void *> ptrs;
  explicit Scratch(tlrqmc_ctx *c) : ctx(c) {}
  ~Scratch() {
    for (void *p : ptrs) ctx->dfree(p);
  }
  template <class T>
  T *get(size_t count) {
    if (count == 0) count = 1;
    void *p = ctx->dmalloc(count * sizeof(T));
    if (p) ptrs.push_back(p);
    return static_cast<T *>(p);
  }
};

// HIP events around launches, summed per kernel kind.
struct Profiler {
  bool on;
  hipStream_t stream;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> marks;
  int open_kind = -1;
  hipEvent_t open_ev = nullptr;
  Profiler(bool enable, hipStream_t s) : on(enable), stream(s) {}
  ~Profiler() {
    for (auto &m : marks) {
      hipEventDestroy(m.second.first);
      hipEventDestroy(m.second.second);
    }
  }
  void begin(int kind) {
    if (!on) return;
    hipEventCreate(&open_ev);
    hipEventRecord(open_ev, stream);
    open_kind = kind;
  }
  void end() {
    if (!on) return;
    hipEvent_t e;
    hipEventCreate(&e);
    hipEventRecord(e, stream);
    marks.push_back({open_kind, {open_ev, e}});
  }
  void collect(tlrqmc_result *r) {
    for (int k = 0; k < TLRQMC_KERNEL_KINDS; ++k) {
      r->kernel_seconds[k] = 0.0;
      r->kernel_launches[k] = 0;
    }
    for (auto &m : marks) {
      float ms = 0.f;
      hipEventElapsedTime(&ms, m.second.first, m.second.second);
      r->kernel_seconds[m.first] += ms * 1e-3;
      r->kernel_launches[m.first] += 1;
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

void finish_estimate(const std::vector<double> &part, int M, int64_t N, tlrqmc_result *out) {
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

// Shared driver of mvn_prob, mvt_prob and tlrqmc_sample_logp.  Samples
// g0 .. g0+count-1 of the flattened (shift, k) index space are swept; a
// full estimate (reduce = true) needs g0 = 0 and count = N M.
int run_estimator(tlrqmc_ctx *ctx, const tlrqmc_factor *f, const double *a, const double *b,
                  double nu, const tlrqmc_qmc_opts *opts, int64_t g0, int64_t count,
                  bool reduce, double *logp_host, tlrqmc_result *out) {
  clear_error();
  if (!ctx || !f || !a || !b || !opts) return fail(TLRQMC_EINVAL, "null argument");
  if (f->ctx != ctx) return fail(TLRQMC_EINVAL, "factor belongs to another context");
  const int64_t N = opts->n_samples;
  const int M = opts->n_shifts;
  if (N < 1) return fail(TLRQMC_EINVAL, "n_samples must be >= 1");
  if (M < 2 || M > 64) return fail(TLRQMC_EINVAL, "n_shifts must be in [2, 64]");
  if (opts->precision != 0 && opts->precision != 1) return fail(TLRQMC_EINVAL, "precision must be 0 or 1");
  if (opts->precision == 1) return fail(TLRQMC_EINVAL, "precision form 1 is not available in this build");
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
      finish_estimate(part, M, N, out);
    }
    return TLRQMC_OK;
  }
  // chunking: Z (k_tot rows) + Y + Delta (padded tile rows) per sample
  const int64_t mpad = round_up(f->m, 64);
  const int64_t per_sample = 8 * (f->k_tot + 2 * mpad + 2);
  int64_t chunk = opts->chunk_samples;
  if (chunk <= 0) {
    const int64_t budget = int64_t{40} << 30;
    chunk = std::max<int64_t>(256, budget / per_sample);
  }
  chunk = round_up(std::min(chunk, count), 256);
  const int64_t ld = chunk;
  Scratch sc(ctx);
  double *d_a = two_sided ? sc.get<double>(n) : nullptr;
  double *d_b = sc.get<double>(n);
  uint64_t *d_D = sc.get<uint64_t>(static_cast<size_t>(M) * (n + 1));
  double *d_logp = sc.get<double>(count);
  double *d_R = nu > 0 ? sc.get<double>(chunk) : nullptr;
  double *d_Y = sc.get<double>(static_cast<size_t>(mpad) * ld);
  double *d_Dl = r > 1 ? sc.get<double>(static_cast<size_t>(mpad) * ld) : nullptr;
  double *d_Z = f->k_tot > 0 ? sc.get<double>(static_cast<size_t>(f->k_tot) * ld) : nullptr;
  double *d_part = reduce ? sc.get<double>(3 * M) : nullptr;
  if (!d_b || !d_D || !d_logp || !d_Y || (two_sided && !d_a) || (nu > 0 && !d_R) ||
      (r > 1 && !d_Dl) || (f->k_tot > 0 && !d_Z) || (reduce && !d_part))
    return fail(TLRQMC_ENOMEM, "device allocation failed (chunk of %lld samples)", static_cast<long long>(chunk));
  const std::vector<uint64_t> shifts = splitmix64_table(opts->seed, static_cast<int64_t>(M) * (n + 1));
  hipStream_t st = ctx->stream;
  if (two_sided && hipMemcpyAsync(d_a, ap.data(), n * 8, hipMemcpyHostToDevice, st) != hipSuccess)
    return fail(TLRQMC_EDEVICE, "copy of limits failed");
  if (hipMemcpyAsync(d_b, bp.data(), n * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(d_D, shifts.data(), shifts.size() * 8, hipMemcpyHostToDevice, st) != hipSuccess)
    return fail(TLRQMC_EDEVICE, "copy of limits or shifts failed");
  hipEvent_t ev0, ev1;
  hipEventCreate(&ev0);
  hipEventCreate(&ev1);
  Profiler prof(opts->profile != 0, st);
  hipEventRecord(ev0, st);
  int chunks = 0;
  for (int64_t c0 = 0; c0 < count; c0 += chunk) {
    const int64_t cnt = std::min(chunk, count - c0);
    ++chunks;
    InitParams ip{g0 + c0, cnt, N, f->d_gen, d_D, n + 1, nu, d_logp + c0, d_R};
    prof.begin(TLRQMC_KERNEL_INIT);
    launch_init(st, ip);
    prof.end();
    if (!check_launch("init")) goto fail_dev;
    for (int j = 0; j < r; ++j) {
      if (j > 0 && f->krow[j] > 0) {
        LrParams lp{cnt, ld, f->tm[j], static_cast<int>(f->krow[j]), f->urow_ld[j],
                    f->d_urow + f->urow_off[j], d_Z + f->zoff[j] * ld, d_Dl, nullptr};
        prof.begin(TLRQMC_KERNEL_DELTA);
        launch_delta_f64(st, lp);
        prof.end();
        if (!check_launch("delta")) goto fail_dev;
      }
      SweepParams sp{g0 + c0, cnt, N, ld, n + 1, f->tm[j], static_cast<int>(1 + f->toff[j]),
                     f->d_diag + f->diag_off[j], two_sided ? d_a + f->toff[j] : nullptr,
                     d_b + f->toff[j], (j > 0 && f->krow[j] > 0) ? d_Dl : nullptr, d_R,
                     f->d_gen, d_D, d_logp + c0, d_Y};
      prof.begin(TLRQMC_KERNEL_SWEEP);
      launch_sweep(st, sp, two_sided, nu > 0);
      prof.end();
      if (!check_launch("sweep")) goto fail_dev;
      if (j < r - 1 && f->kcol[j] > 0) {
        LrParams lp{cnt, ld, static_cast<int>(f->kcol[j]), f->tm[j], f->vpan_ld[j],
                    f->d_vpan + f->vpan_off[j], d_Y, d_Z, f->d_zmap + f->zmap_off[j]};
        prof.begin(TLRQMC_KERNEL_ZPROJ);
        launch_zproj_f64(st, lp);
        prof.end();
        if (!check_launch("zproj")) goto fail_dev;
      }
    }
  }
  if (reduce) {
    ReduceParams rp{N, d_logp, d_part};
    prof.begin(TLRQMC_KERNEL_REDUCE);
    launch_reduce(st, rp, M);
    prof.end();
    if (!check_launch("reduce")) goto fail_dev;
  }
  hipEventRecord(ev1, st);
  {
    std::vector<double> part(reduce ? 3 * M : 0);
    if (reduce && hipMemcpyAsync(part.data(), d_part, part.size() * 8, hipMemcpyDeviceToHost, st) != hipSuccess)
      goto fail_dev;
    if (logp_host && hipMemcpyAsync(logp_host, d_logp, count * 8, hipMemcpyDeviceToHost, st) != hipSuccess)
      goto fail_dev;
    if (hipStreamSynchronize(st) != hipSuccess) goto fail_dev;
    float ms = 0.f;
    hipEventElapsedTime(&ms, ev0, ev1);
    hipEventDestroy(ev0);
    hipEventDestroy(ev1);
    if (out) {
      if (reduce) finish_estimate(part, M, N, out);
      out->seconds = ms * 1e-3;
      out->chunks = chunks;
      prof.collect(out);
    }
  }
  return TLRQMC_OK;
fail_dev:
  hipStreamSynchronize(st);
  hipEventDestroy(ev0);
  hipEventDestroy(ev1);
  if (tlrqmc_last_error()[0] == '\0') fail(TLRQMC_EDEVICE, "HIP error: %s", hipGetErrorString(hipGetLastError()));
  return TLRQMC_EDEVICE;
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

void tlrqmc_ctx::dfree(void *p) {
  if (!p) return;
  if (has_alloc) alloc.free(p, alloc.user);
  else hipFree(p);
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

void tlrqmc_ctx_destroy(tlrqmc_ctx *ctx) { delete ctx; }

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
    hipSetDevice(f->ctx->device);
    hipStreamSynchronize(f->ctx->stream);
    f->ctx->dfree(f->d_diag);
    f->ctx->dfree(f->d_urow);
    f->ctx->dfree(f->d_vpan);
    f->ctx->dfree(f->d_zmap);
    f->ctx->dfree(f->d_gen);
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

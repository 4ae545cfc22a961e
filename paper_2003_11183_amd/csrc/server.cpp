// Request server: continuous batching of probability requests on one GPU.
//
// A request is one probability of its own dimension, covariance and limits
// (the likelihood of Section 5 asks for many of them).  Its life:
//   queued  -> admitted to setup when its reservation fits the budget
//   setup   -> ordering (geometric or block reordering, Section 3.3) and
//              the TLR factor (Section 3.3), on the setup thread and stream
//   ready   -> its samples are cut into slots of a size fixed by the
//              request alone; slots become active as memory allows
//   running -> every step advances every active slot, of every request, by
//              one diagonal tile (Section 3.4) in shared batched launches
//   done    -> per-shift reduction and the estimate (Section 2.1)
// The samples of a slot see exactly the arithmetic of the single-request
// path, and the reduction of a request runs over its own samples in a fixed
// order, so a result does not depend on the other requests in flight.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include <omp.h>

#include "internal.hpp"
#include "setup_kernels.hpp"

namespace tlrqmc {

namespace {

using Clock = std::chrono::steady_clock;

// Active slots per step (descriptor capacity of one step).
constexpr int kMaxSlots = 64;
// Requests set up concurrently: one's device work (Cholesky, compression)
// overlaps the host ordering and layout of the others.
constexpr int kSetupWorkers = 6;
constexpr int64_t kAlign = 256;

// Device arena: one allocation from the caller's allocator, carved by best
// fit with coalescing of neighbouring holes.
class Arena {
 public:
  bool init(tlrqmc_ctx *ctx, size_t bytes) {
    cap_ = static_cast<size_t>(round_up(static_cast<int64_t>(bytes), kAlign));
    base_ = static_cast<char *>(ctx->dmalloc(cap_));
    if (!base_) return false;
    holes_[0] = cap_;
    return true;
  }
  void release(tlrqmc_ctx *ctx) {
    if (base_) ctx->dfree(base_);
    base_ = nullptr;
  }
  void *alloc(size_t bytes) {
    std::lock_guard<std::mutex> g(mu_);
    const size_t need = static_cast<size_t>(round_up(static_cast<int64_t>(bytes ? bytes : 1), kAlign));
    auto best = holes_.end();
    for (auto it = holes_.begin(); it != holes_.end(); ++it)
      if (it->second >= need && (best == holes_.end() || it->second < best->second)) best = it;
    if (best == holes_.end()) return nullptr;
    const size_t off = best->first, size = best->second;
    holes_.erase(best);
    if (size > need) holes_[off + need] = size - need;
    used_[off] = need;
    in_use_ += need;
    peak_ = std::max(peak_, in_use_);
    return base_ + off;
  }
  void free(void *p) {
    if (!p) return;
    std::lock_guard<std::mutex> g(mu_);
    const size_t off = static_cast<size_t>(static_cast<char *>(p) - base_);
    auto u = used_.find(off);
    if (u == used_.end()) return;
    size_t start = off, size = u->second;
    in_use_ -= size;
    used_.erase(u);
    auto next = holes_.lower_bound(start);
    if (next != holes_.end() && next->first == start + size) {
      size += next->second;
      next = holes_.erase(next);
    }
    if (next != holes_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        start = prev->first;
        size += prev->second;
        holes_.erase(prev);
      }
    }
    holes_[start] = size;
  }
  size_t in_use() {
    std::lock_guard<std::mutex> g(mu_);
    return in_use_;
  }
  size_t peak() {
    std::lock_guard<std::mutex> g(mu_);
    return peak_;
  }
  size_t capacity() const { return cap_; }

 private:
  std::mutex mu_;
  char *base_ = nullptr;
  size_t cap_ = 0, in_use_ = 0, peak_ = 0;
  std::map<size_t, size_t> holes_, used_;
};

void *arena_alloc(size_t bytes, void *user) { return static_cast<Arena *>(user)->alloc(bytes); }
void arena_free(void *p, void *user) { static_cast<Arena *>(user)->free(p); }

enum State { QUEUED, SETUP, READY, RUNNING, DONE };

struct Request {
  uint64_t id = 0;
  // copied inputs
  int64_t n = 0;
  tlrqmc_cov cov{};
  std::vector<double> xy, sigma, a, b;
  double nu = 0.0;
  int m = 0, max_rank = 0, reorder = 0;
  double tol = 0.0;
  tlrqmc_qmc_opts qmc{};
  // lifecycle
  State state = QUEUED;
  int status = TLRQMC_OK;
  std::string error;
  tlrqmc_result result{};
  tlrqmc_request_info info{};
  int64_t reserve = 0;      // bytes of the budget held for this request
  std::vector<uint64_t> shifts;
  // setup output
  tlrqmc_factor *f = nullptr;
  int factor_status = TLRQMC_OK;
  // run plan
  bool two_sided = false, scaled = false, prec = false;
  int64_t count = 0, chunk = 0, slot_bytes = 0, req_bytes = 0;
  int nslots = 0, concurrency = 1, started = 0, active = 0, finished = 0;
  std::vector<double> ap, bp;
  double *d_a = nullptr, *d_b = nullptr, *d_logp = nullptr, *d_part = nullptr;
  uint64_t *d_D = nullptr;
  double *h_part = nullptr;  // pinned
  bool reduced = false;
};

struct Slot {
  Request *q = nullptr;
  int64_t c0 = 0, cnt = 0;
  int j = 0;
  ChunkBuffers b;
};

// Descriptors of one step, grouped by kernel variant.
struct StepBatch {
  std::vector<InitParams> init;
  int64_t init_max = 0;
  std::vector<MfmaLrParams> lr[2][2];  // [delta, projection][row tiles 1, 2]
  int64_t lr_max[2][2] = {};
  std::vector<LrParams> f64[2];        // [delta, projection]
  int64_t f64_max[2] = {};
  int f64_rows[2] = {};
  std::vector<SweepParams> sweep[8];   // two_sided * 4 + scaled * 2 + prec
  int64_t sweep_max[8] = {};
  std::vector<ReduceParams> reduce;
  int reduce_max = 0;
  void clear() {
    init.clear();
    init_max = 0;
    for (auto &k : lr)
      for (auto &v : k) v.clear();
    std::memset(lr_max, 0, sizeof lr_max);
    for (auto &v : f64) v.clear();
    f64_max[0] = f64_max[1] = 0;
    f64_rows[0] = f64_rows[1] = 0;
    for (auto &v : sweep) v.clear();
    std::memset(sweep_max, 0, sizeof sweep_max);
    reduce.clear();
    reduce_max = 0;
  }
};

int rt_index(int rt) { return rt - 1; }

}  // namespace
}  // namespace tlrqmc

using namespace tlrqmc;

struct tlrqmc_server {
  tlrqmc_ctx *user = nullptr;
  Arena arena;
  tlrqmc_ctx sctx[kSetupWorkers], rctx;  // setup and run contexts on the arena
  size_t budget = 0;
  Clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv;
  std::map<uint64_t, std::unique_ptr<Request>> reqs;
  std::deque<Request *> queued, ready;
  int64_t reserved = 0;
  int64_t peak_reserved = 0;
  bool stop = false;
  uint64_t next_id = 1;
  int in_setup = 0, in_run = 0;
  // step thread state
  std::vector<Slot> slots;
  std::vector<Request *> running;
  int64_t steps = 0, launches = 0, slot_steps = 0, max_active = 0;
  // per-step staging: two pinned host buffers and two device buffers
  char *h_desc[2] = {nullptr, nullptr};
  char *d_desc[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool ev_pending[2] = {false, false};
  std::vector<void *> defer_free[2];
  std::vector<Request *> defer_done[2];
  size_t desc_bytes = 0;
  std::thread t_setup[kSetupWorkers], t_run;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
  void setup_loop(int w);
  void run_loop();
  bool plan(Request *q);
  bool start_request(Request *q);
  bool activate_slot(Request *q);
  void complete(Request *q);
  void fail_request(Request *q, int code, const std::string &msg);
  void release(Request *q);
  void retire(int which);
  int step(StepBatch &B, int cur);
};

namespace tlrqmc {
namespace {

// Device bytes of setup: the dense covariance (leading dimension padded to
// 64), the locations and the tile compression's batch buffers, plus slack
// for the factor's small arrays.
int64_t setup_reserve(int64_t n, int m) {
  return 8 * round_up(n, 64) * n + 64 * n + compress_scratch_bytes(n, m) + (int64_t{1} << 20);
}

}  // namespace
}  // namespace tlrqmc

// Called with mu held.
void tlrqmc_server::fail_request(Request *q, int code, const std::string &msg) {
  q->status = code;
  q->error = msg;
  q->state = DONE;
  q->info.t_done = now();
  q->info.status = code;
  cv.notify_all();
}

// Free what a request holds and return its reservation (mu held; the
// device has finished with every buffer).
void tlrqmc_server::release(Request *q) {
  for (void *p : {static_cast<void *>(q->d_a), static_cast<void *>(q->d_b), static_cast<void *>(q->d_D),
                  static_cast<void *>(q->d_logp), static_cast<void *>(q->d_part)})
    arena.free(p);
  q->d_a = q->d_b = q->d_logp = q->d_part = nullptr;
  q->d_D = nullptr;
  if (q->h_part) (void)hipHostFree(q->h_part);
  q->h_part = nullptr;
  if (q->f) tlrqmc_factor_free(q->f);
  q->f = nullptr;
  reserved -= q->reserve;
  q->reserve = 0;
  std::vector<double>().swap(q->xy);
  std::vector<double>().swap(q->sigma);
  std::vector<uint64_t>().swap(q->shifts);
}

void tlrqmc_server::setup_loop(int w) {
  (void)hipSetDevice(user->device);
  // this worker's share of the host threads for its parallel loops
  omp_set_num_threads(std::max(1, omp_get_num_procs() / kSetupWorkers));
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv.wait(lk, [&] {
      if (queued.empty()) return stop;
      const int64_t need = setup_reserve(queued.front()->n, queued.front()->m);
      return need > static_cast<int64_t>(budget) || reserved + need <= static_cast<int64_t>(budget);
    });
    if (queued.empty()) return;
    Request *q = queued.front();
    queued.pop_front();
    if (setup_reserve(q->n, q->m) > static_cast<int64_t>(budget)) {
      fail_request(q, TLRQMC_ENOMEM,
                   "setup of the request needs " + std::to_string(setup_reserve(q->n, q->m)) +
                       " bytes of device memory, more than the server budget");
      continue;
    }
    q->reserve = setup_reserve(q->n, q->m);
    reserved += q->reserve;
    peak_reserved = std::max(peak_reserved, reserved);
    q->state = SETUP;
    q->info.t_admit = now();
    ++in_setup;
    lk.unlock();
    int st = TLRQMC_OK;
    std::string msg;
    std::vector<int32_t> perm;
    tlrqmc_factor *f = nullptr;
    for (int attempt = 0;; ++attempt) {
      st = TLRQMC_OK;
      if (q->reorder) {
        perm.resize(q->n);
        st = block_reorder(nullptr, q->n, &q->cov, q->a.data(), q->b.data(), q->m, perm.data());
      }
      if (st == TLRQMC_OK)
        st = tlr_factor(&sctx[w], q->n, &q->cov, q->reorder ? perm.data() : nullptr, q->m, q->tol, q->max_rank, &f);
      if (st < 0) msg = tlrqmc_last_error();
      // The arena may be fragmented by slots in flight: wait for frees.
      if (st != TLRQMC_ENOMEM || attempt >= 500) break;
      lk.lock();
      const bool idle = running.empty() && slots.empty();
      cv.wait_for(lk, std::chrono::milliseconds(20));
      lk.unlock();
      if (idle && attempt > 10) break;
    }
    lk.lock();
    --in_setup;
    if (st < 0) {
      reserved -= q->reserve;
      q->reserve = 0;
      fail_request(q, st, msg);
      continue;
    }
    q->f = f;
    q->factor_status = st;
    q->info.t_ready = now();
    if (!plan(q)) continue;
    q->state = READY;
    ready.push_back(q);
    cv.notify_all();
  }
}

// Slot size, buffers and concurrency of a request after setup (mu held).
// The reservation becomes the footprint of all its slots at once, capped at
// the larger of its setup reservation and a quarter of the budget, but at
// least one slot's; it may exceed the budget for a while, which holds back
// new setups until running requests return memory.
bool tlrqmc_server::plan(Request *q) {
  tlrqmc_factor *f = q->f;
  q->prec = q->qmc.precision == 1;
  q->scaled = q->nu > 0.0;
  q->ap.resize(q->n);
  q->bp.resize(q->n);
  for (int64_t i = 0; i < q->n; ++i) {
    q->ap[i] = q->a[f->perm[i]];
    q->bp[i] = q->b[f->perm[i]];
    if (q->ap[i] > -INFINITY) q->two_sided = true;
  }
  const int64_t M = q->qmc.n_shifts, N = q->qmc.n_samples;
  q->count = N * M;
  auto al = [](int64_t b) { return round_up(b, kAlign); };
  const SlotPlan sp = plan_slots(f, q->prec, q->scaled, q->count);
  q->chunk = sp.chunk;
  q->nslots = sp.nslots;
  q->slot_bytes = sp.slot_bytes;
  q->req_bytes = al(8 * q->n) * (q->two_sided ? 2 : 1) + al(8 * M * (q->n + 1)) + al(8 * q->count) + al(8 * 3 * M);
  const int64_t fixed = f->device_bytes + q->req_bytes;
  const int64_t f_min = fixed + q->slot_bytes, f_all = fixed + q->nslots * q->slot_bytes;
  if (f_min > static_cast<int64_t>(budget)) {
    reserved -= q->reserve;
    q->reserve = 0;
    tlrqmc_factor_free(q->f);
    q->f = nullptr;
    fail_request(q, TLRQMC_ENOMEM,
                 "request needs " + std::to_string(f_min) + " bytes of device memory, more than the server budget");
    return false;
  }
  const int64_t want = std::max(f_min, std::min(f_all, std::max(q->reserve, static_cast<int64_t>(budget / 4))));
  reserved += want - q->reserve;
  q->reserve = want;
  peak_reserved = std::max(peak_reserved, reserved);
  q->concurrency = static_cast<int>(std::min<int64_t>(q->nslots, (want - fixed) / q->slot_bytes));
  q->info.slots = q->nslots;
  q->info.concurrency = q->concurrency;
  q->info.chunk_samples = q->chunk;
  q->info.reserved_bytes = want;
  q->info.factor_bytes = f->device_bytes;
  q->info.factor_checksum = f->checksum;
  return true;
}

// Request buffers, limits and shifts on the device (mu held).
bool tlrqmc_server::start_request(Request *q) {
  const int64_t n = q->n, M = q->qmc.n_shifts;
  q->d_b = static_cast<double *>(arena.alloc(8 * n));
  q->d_a = q->two_sided ? static_cast<double *>(arena.alloc(8 * n)) : nullptr;
  q->d_D = static_cast<uint64_t *>(arena.alloc(8 * M * (n + 1)));
  q->d_logp = static_cast<double *>(arena.alloc(8 * q->count));
  q->d_part = static_cast<double *>(arena.alloc(8 * 3 * M));
  void *hp = nullptr;
  const bool ok = q->d_b && (!q->two_sided || q->d_a) && q->d_D && q->d_logp && q->d_part &&
                  hipHostMalloc(&hp, 8 * 3 * M, hipHostMallocDefault) == hipSuccess;
  q->h_part = static_cast<double *>(hp);
  if (!ok) {
    for (void *p : {static_cast<void *>(q->d_a), static_cast<void *>(q->d_b), static_cast<void *>(q->d_D),
                    static_cast<void *>(q->d_logp), static_cast<void *>(q->d_part)})
      arena.free(p);
    q->d_a = q->d_b = q->d_logp = q->d_part = nullptr;
    q->d_D = nullptr;
    if (q->h_part) (void)hipHostFree(q->h_part);
    q->h_part = nullptr;
    return false;
  }
  q->shifts = splitmix64_table(q->qmc.seed, M * (n + 1));
  hipStream_t s = rctx.stream;
  bool cp = hipMemcpyAsync(q->d_b, q->bp.data(), 8 * n, hipMemcpyHostToDevice, s) == hipSuccess &&
            hipMemcpyAsync(q->d_D, q->shifts.data(), 8 * M * (n + 1), hipMemcpyHostToDevice, s) == hipSuccess;
  if (q->two_sided) cp = cp && hipMemcpyAsync(q->d_a, q->ap.data(), 8 * n, hipMemcpyHostToDevice, s) == hipSuccess;
  if (!cp) {
    fail_request(q, TLRQMC_EDEVICE, "copy of a request's limits failed");
    return true;
  }
  q->state = RUNNING;
  return true;
}

// Buffers of the next slot of q (mu held); false when the arena is full.
bool tlrqmc_server::activate_slot(Request *q) {
  Slot s;
  s.q = q;
  s.c0 = static_cast<int64_t>(q->started) * q->chunk;
  s.cnt = std::min(q->chunk, q->count - s.c0);
  std::vector<void *> got;
  int64_t bytes[4];
  chunk_buffer_bytes(q->f, q->prec, q->scaled, q->chunk, bytes);
  void *b[4] = {nullptr, nullptr, nullptr, nullptr};
  for (int k = 0; k < 4; ++k)
    if (bytes[k] > 0) got.push_back(b[k] = arena.alloc(bytes[k]));
  s.b.Y = b[0];
  s.b.R = static_cast<double *>(b[3]);
  if (q->prec) {
    s.b.DlF = static_cast<float *>(b[1]);
    s.b.ZF = static_cast<float *>(b[2]);
  } else {
    s.b.Dl = static_cast<double *>(b[1]);
    s.b.Z = static_cast<double *>(b[2]);
  }
  for (void *p : got)
    if (!p) {
      for (void *x : got) arena.free(x);
      return false;
    }
  if (q->started == 0) q->info.t_start = now();
  ++q->started;
  ++q->active;
  slots.push_back(s);
  return true;
}

// Estimate of a finished request (mu held; its partial sums are on the host).
void tlrqmc_server::complete(Request *q) {
  const int M = q->qmc.n_shifts;
  std::vector<double> part(q->h_part, q->h_part + 3 * M);
  estimate_from_parts(part, M, q->qmc.n_samples, &q->result);
  q->result.chunks = q->nslots;
  release(q);
  q->state = DONE;
  q->status = q->factor_status;
  q->info.t_done = now();
  q->info.status = q->status;
  q->result.seconds = q->info.t_done - q->info.t_submit;
  cv.notify_all();
}

// Frees and completions of a finished step (mu held).
void tlrqmc_server::retire(int which) {
  for (void *p : defer_free[which]) arena.free(p);
  defer_free[which].clear();
  for (Request *q : defer_done[which]) complete(q);
  defer_done[which].clear();
  ev_pending[which] = false;
}

// Build, upload and launch one step on staging buffer `cur`; returns a
// HIP status (0 = launched).
int tlrqmc_server::step(StepBatch &B, int cur) {
  B.clear();
  std::vector<Request *> finishing;
  std::vector<Slot> keep;
  keep.reserve(slots.size());
  for (Slot &s : slots) {
    Request *q = s.q;
    const tlrqmc_factor *f = q->f;
    const int j = s.j, r = f->r;
    const int64_t ld = q->chunk, N = q->qmc.n_samples;
    const ChunkRun run{s.c0, s.cnt, N, ld, q->prec, s.b, q->d_a, q->d_b, q->d_D, q->d_logp + s.c0};
    if (j == 0) {
      B.init.push_back(init_launch(f, run, q->nu));
      B.init_max = std::max(B.init_max, s.cnt);
    }
    const TileLaunch t = tile_launch(f, j, run);
    if (t.delta) {
      if (q->prec) {
        const int k = rt_index(lr_mfma_rt(t.delta_mfma.rows));
        B.lr[0][k].push_back(t.delta_mfma);
        B.lr_max[0][k] = std::max(B.lr_max[0][k], lr_mfma_blocks(s.cnt, t.delta_mfma.rows));
      } else {
        B.f64[0].push_back(t.delta_f64);
        B.f64_max[0] = std::max(B.f64_max[0], s.cnt);
        B.f64_rows[0] = std::max(B.f64_rows[0], t.delta_f64.rows);
      }
    }
    const int v = (q->two_sided ? 4 : 0) + (q->scaled ? 2 : 0) + (q->prec ? 1 : 0);
    B.sweep[v].push_back(t.sweep);
    B.sweep_max[v] = std::max(B.sweep_max[v], s.cnt);
    if (t.zproj) {
      if (q->prec) {
        const int k = rt_index(lr_mfma_rt(t.zproj_mfma.rows));
        B.lr[1][k].push_back(t.zproj_mfma);
        B.lr_max[1][k] = std::max(B.lr_max[1][k], lr_mfma_blocks(s.cnt, t.zproj_mfma.rows));
      } else {
        B.f64[1].push_back(t.zproj_f64);
        B.f64_max[1] = std::max(B.f64_max[1], s.cnt);
        B.f64_rows[1] = std::max(B.f64_rows[1], t.zproj_f64.rows);
      }
    }
    ++slot_steps;
    if (++s.j < r) {
      keep.push_back(s);
      continue;
    }
    // slot finished: its buffers are free once this step has run
    for (void *p : {s.b.Y, static_cast<void *>(s.b.Dl), static_cast<void *>(s.b.Z), static_cast<void *>(s.b.R),
                    static_cast<void *>(s.b.DlF), static_cast<void *>(s.b.ZF)})
      if (p) defer_free[cur].push_back(p);
    --q->active;
    if (++q->finished == q->nslots) {
      B.reduce.push_back(ReduceParams{N, q->qmc.n_shifts, q->d_logp, q->d_part});
      B.reduce_max = std::max(B.reduce_max, q->qmc.n_shifts);
      finishing.push_back(q);
    }
  }
  slots.swap(keep);
  // stage descriptors
  size_t off = 0;
  char *h = h_desc[cur];
  auto stage = [&](const void *src, size_t bytes) {
    const size_t at = off;
    if (at + bytes <= desc_bytes && bytes) std::memcpy(h + at, src, bytes);
    off = static_cast<size_t>(round_up(static_cast<int64_t>(at + bytes), 256));
    return at;
  };
  const size_t o_init = stage(B.init.data(), B.init.size() * sizeof(InitParams));
  size_t o_lr[2][2], o_f64[2], o_sw[8];
  for (int k = 0; k < 2; ++k)
    for (int t = 0; t < 2; ++t) o_lr[k][t] = stage(B.lr[k][t].data(), B.lr[k][t].size() * sizeof(MfmaLrParams));
  for (int k = 0; k < 2; ++k) o_f64[k] = stage(B.f64[k].data(), B.f64[k].size() * sizeof(LrParams));
  for (int v = 0; v < 8; ++v) o_sw[v] = stage(B.sweep[v].data(), B.sweep[v].size() * sizeof(SweepParams));
  const size_t o_red = stage(B.reduce.data(), B.reduce.size() * sizeof(ReduceParams));
  if (off > desc_bytes) return 5;  // cannot happen with kMaxSlots slots
  // kernel launches: no library factorization (setup workers) runs beside them
  SharedDevice dev;
  hipStream_t st = rctx.stream;
  char *d = d_desc[cur];
  if (hipMemcpyAsync(d, h, off, hipMemcpyHostToDevice, st) != hipSuccess) return 1;
  int nl = 0;
  if (!B.init.empty()) {
    launch_init_batch(st, reinterpret_cast<const InitParams *>(d + o_init), static_cast<int>(B.init.size()), B.init_max);
    ++nl;
  }
  for (int t = 0; t < 2; ++t)
    if (!B.lr[0][t].empty()) {
      launch_lr_mfma_batch(st, reinterpret_cast<const MfmaLrParams *>(d + o_lr[0][t]),
                           static_cast<int>(B.lr[0][t].size()), t + 1, false, false, B.lr_max[0][t]);
      ++nl;
    }
  if (!B.f64[0].empty()) {
    launch_delta_f64_batch(st, reinterpret_cast<const LrParams *>(d + o_f64[0]), static_cast<int>(B.f64[0].size()),
                           B.f64_max[0], B.f64_rows[0]);
    ++nl;
  }
  for (int v = 0; v < 8; ++v)
    if (!B.sweep[v].empty()) {
      launch_sweep_batch(st, reinterpret_cast<const SweepParams *>(d + o_sw[v]), static_cast<int>(B.sweep[v].size()),
                         B.sweep_max[v], (v & 4) != 0, (v & 2) != 0, (v & 1) != 0);
      ++nl;
    }
  for (int t = 0; t < 2; ++t)
    if (!B.lr[1][t].empty()) {
      launch_lr_mfma_batch(st, reinterpret_cast<const MfmaLrParams *>(d + o_lr[1][t]),
                           static_cast<int>(B.lr[1][t].size()), t + 1, false, true, B.lr_max[1][t]);
      ++nl;
    }
  if (!B.f64[1].empty()) {
    launch_zproj_f64_batch(st, reinterpret_cast<const LrParams *>(d + o_f64[1]), static_cast<int>(B.f64[1].size()),
                           B.f64_max[1], B.f64_rows[1]);
    ++nl;
  }
  if (!B.reduce.empty()) {
    launch_reduce_batch(st, reinterpret_cast<const ReduceParams *>(d + o_red), static_cast<int>(B.reduce.size()),
                        B.reduce_max);
    ++nl;
  }
  if (hipGetLastError() != hipSuccess) return 2;
  for (Request *q : finishing) {
    if (hipMemcpyAsync(q->h_part, q->d_part, 8 * 3 * q->qmc.n_shifts, hipMemcpyDeviceToHost, st) != hipSuccess)
      return 3;
    defer_done[cur].push_back(q);
    running.erase(std::find(running.begin(), running.end(), q));
  }
  if (hipEventRecord(ev[cur], st) != hipSuccess) return 4;
  ev_pending[cur] = true;
  ++steps;
  launches += nl;
  return 0;
}

void tlrqmc_server::run_loop() {
  (void)hipSetDevice(user->device);
  StepBatch B;
  int cur = 0;
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    // start ready requests in arrival order, then activate their slots
    while (!ready.empty()) {
      Request *q = ready.front();
      if (!start_request(q)) break;
      ready.pop_front();
      if (q->state == RUNNING) running.push_back(q);
      else release(q);
    }
    for (Request *q : running)
      while (q->started < q->nslots && q->active < q->concurrency && static_cast<int>(slots.size()) < kMaxSlots)
        if (!activate_slot(q)) break;
    max_active = std::max<int64_t>(max_active, static_cast<int64_t>(slots.size()));
    if (slots.empty()) {
      if (ev_pending[0] || ev_pending[1]) {
        lk.unlock();
        (void)hipStreamSynchronize(rctx.stream);
        lk.lock();
        for (int k = 0; k < 2; ++k)
          if (ev_pending[k]) retire(k);
        continue;
      }
      if (stop && queued.empty() && ready.empty() && in_setup == 0 && running.empty()) return;
      cv.notify_all();
      // nothing to run: wait for a ready request, or for memory when one
      // is waiting
      if (!ready.empty() || !running.empty()) cv.wait_for(lk, std::chrono::milliseconds(5));
      else cv.wait(lk, [&] { return !ready.empty() || (stop && queued.empty() && in_setup == 0); });
      continue;
    }
    const int rc = step(B, cur);
    if (rc != 0) {
      // a failed launch or copy: fail everything in flight on this server
      const std::string msg = std::string("HIP error in a serving step: ") + hipGetErrorString(hipGetLastError());
      lk.unlock();
      (void)hipStreamSynchronize(rctx.stream);
      lk.lock();
      for (Slot &s : slots) s.q->active = 0;
      slots.clear();
      for (int k = 0; k < 2; ++k) {
        for (void *p : defer_free[k]) arena.free(p);
        defer_free[k].clear();
        for (Request *q : defer_done[k]) {
          release(q);
          fail_request(q, TLRQMC_EDEVICE, msg);
        }
        defer_done[k].clear();
        ev_pending[k] = false;
      }
      for (Request *q : running) {
        release(q);
        fail_request(q, TLRQMC_EDEVICE, msg);
      }
      running.clear();
      continue;
    }
    // keep at most two steps in flight: wait for the previous one
    const int prev = cur ^ 1;
    if (ev_pending[prev]) {
      lk.unlock();
      (void)hipEventSynchronize(ev[prev]);
      lk.lock();
      retire(prev);
    }
    cur = prev;
  }
}

extern "C" {

int tlrqmc_server_create(tlrqmc_ctx *ctx, size_t hbm_budget_bytes, tlrqmc_server **out) {
  clear_error();
  if (!ctx || !out) return fail(TLRQMC_EINVAL, "null argument");
  if (hbm_budget_bytes < (size_t{1} << 24)) return fail(TLRQMC_EINVAL, "hbm_budget_bytes must be at least 16 MiB");
  *out = nullptr;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(TLRQMC_EDEVICE, "hipSetDevice failed");
  std::unique_ptr<tlrqmc_server> s(new tlrqmc_server());
  s->user = ctx;
  s->budget = hbm_budget_bytes;
  s->t0 = Clock::now();
  if (!s->arena.init(ctx, hbm_budget_bytes))
    return fail(TLRQMC_ENOMEM, "allocation of the %zu-byte server arena failed", hbm_budget_bytes);
  std::vector<tlrqmc_ctx *> all{&s->rctx};
  for (int w = 0; w < kSetupWorkers; ++w) all.push_back(&s->sctx[w]);
  for (tlrqmc_ctx *c : all) {
    c->device = ctx->device;
    c->alloc = tlrqmc_allocator{arena_alloc, arena_free, &s->arena};
    c->has_alloc = true;
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      s->arena.release(ctx);
      return fail(TLRQMC_EDEVICE, "hipStreamCreateWithFlags failed");
    }
  }
  s->desc_bytes = 256 * 1024;
  for (int k = 0; k < 2; ++k) {
    void *h = nullptr;
    s->d_desc[k] = static_cast<char *>(s->arena.alloc(s->desc_bytes));
    if (hipHostMalloc(&h, s->desc_bytes, hipHostMallocDefault) != hipSuccess || !s->d_desc[k] ||
        hipEventCreateWithFlags(&s->ev[k], hipEventDisableTiming) != hipSuccess) {
      if (h) (void)hipHostFree(h);
      for (int i = 0; i < k; ++i) {
        (void)hipHostFree(s->h_desc[i]);
        (void)hipEventDestroy(s->ev[i]);
      }
      for (tlrqmc_ctx *c : all) (void)hipStreamDestroy(c->stream);
      s->arena.release(ctx);
      return fail(TLRQMC_EDEVICE, "allocation of the step staging buffers failed");
    }
    s->h_desc[k] = static_cast<char *>(h);
  }
  tlrqmc_server *srv = s.get();
  for (int w = 0; w < kSetupWorkers; ++w) srv->t_setup[w] = std::thread([srv, w] { srv->setup_loop(w); });
  srv->t_run = std::thread([srv] { srv->run_loop(); });
  *out = s.release();
  return TLRQMC_OK;
}

int tlrqmc_server_submit(tlrqmc_server *s, const tlrqmc_request *req, uint64_t *ticket) {
  clear_error();
  if (!s || !req || !ticket) return fail(TLRQMC_EINVAL, "null argument");
  const int64_t n = req->n;
  if (n < 1) return fail(TLRQMC_EINVAL, "n must be >= 1");
  if (req->m < 1) return fail(TLRQMC_EINVAL, "m must be >= 1");
  if (!req->a || !req->b) return fail(TLRQMC_EINVAL, "a and b are required");
  if (!(req->nu >= 0.0) || std::isinf(req->nu)) return fail(TLRQMC_EINVAL, "nu must be finite and >= 0");
  if (!(req->tol >= 0.0)) return fail(TLRQMC_EINVAL, "tol must be >= 0");
  if (req->max_rank < 0) return fail(TLRQMC_EINVAL, "max_rank must be >= 0");
  const tlrqmc_qmc_opts &o = req->qmc;
  if (o.n_samples < 1) return fail(TLRQMC_EINVAL, "n_samples must be >= 1");
  if (o.n_shifts < 2 || o.n_shifts > 64) return fail(TLRQMC_EINVAL, "n_shifts must be in [2, 64]");
  if (o.precision != 0 && o.precision != 1) return fail(TLRQMC_EINVAL, "precision must be 0 or 1");
  if (o.n_samples > (int64_t{1} << 40) / o.n_shifts) return fail(TLRQMC_EINVAL, "too many samples");
  const tlrqmc_cov &c = req->cov;
  if (c.kind == 1) {
    if (!c.xy || !(c.range > 0.0) || !(c.variance > 0.0) || !(c.nugget >= 0.0))
      return fail(TLRQMC_EINVAL, "exponential covariance needs xy, range > 0, variance > 0, nugget >= 0");
  } else if (c.kind == 0) {
    if (!c.sigma || c.ld < n) return fail(TLRQMC_EINVAL, "dense covariance needs sigma and ld >= n");
  } else {
    return fail(TLRQMC_EINVAL, "unknown covariance kind %d", c.kind);
  }
  std::unique_ptr<Request> q(new Request());
  q->n = n;
  q->cov = c;
  if (c.kind == 1) {
    q->xy.assign(c.xy, c.xy + 2 * n);
    q->cov.xy = q->xy.data();
  } else {
    q->sigma.resize(static_cast<size_t>(n) * n);
    for (int64_t j = 0; j < n; ++j) std::memcpy(&q->sigma[j * n], c.sigma + j * c.ld, 8 * n);
    q->cov.sigma = q->sigma.data();
    q->cov.ld = n;
  }
  q->a.assign(req->a, req->a + n);
  q->b.assign(req->b, req->b + n);
  bool empty = false;
  for (int64_t i = 0; i < n; ++i) {
    if (std::isnan(q->a[i]) || std::isnan(q->b[i])) return fail(TLRQMC_EINVAL, "NaN limit at variable %lld", (long long)i);
    if (q->a[i] >= q->b[i]) empty = true;
  }
  q->nu = req->nu;
  q->m = req->m;
  q->tol = req->tol;
  q->max_rank = req->max_rank;
  q->reorder = req->reorder;
  q->qmc = o;
  q->qmc.logp_out = nullptr;
  std::lock_guard<std::mutex> g(s->mu);
  if (s->stop) return fail(TLRQMC_EINVAL, "server is shutting down");
  q->id = s->next_id++;
  q->info.t_submit = s->now();
  *ticket = q->id;
  Request *raw = q.get();
  s->reqs[q->id] = std::move(q);
  if (empty) {
    // an empty box: probability 0 without touching the device
    const int M = o.n_shifts;
    std::vector<double> part(3 * M, 0.0);
    for (int k = 0; k < M; ++k) {
      part[3 * k] = -INFINITY;
      part[3 * k + 2] = static_cast<double>(o.n_samples);
    }
    estimate_from_parts(part, M, o.n_samples, &raw->result);
    raw->state = DONE;
    raw->info.t_admit = raw->info.t_ready = raw->info.t_start = raw->info.t_done = s->now();
    s->cv.notify_all();
    return TLRQMC_OK;
  }
  s->queued.push_back(raw);
  s->cv.notify_all();
  return TLRQMC_OK;
}

int tlrqmc_server_poll(tlrqmc_server *s, uint64_t ticket, int32_t wait_ms, tlrqmc_result *out,
                       tlrqmc_request_info *info) {
  clear_error();
  if (!s) return fail(TLRQMC_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(TLRQMC_ENOTFOUND, "unknown ticket %llu", static_cast<unsigned long long>(ticket));
  Request *q = it->second.get();
  if (q->state != DONE) {
    if (wait_ms == 0) return TLRQMC_PENDING;
    if (wait_ms < 0) s->cv.wait(lk, [&] { return q->state == DONE; });
    else if (!s->cv.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return q->state == DONE; }))
      return TLRQMC_PENDING;
  }
  if (out) *out = q->result;
  if (info) *info = q->info;
  const int st = q->status;
  if (st < 0) fail(st, "%s", q->error.c_str());
  s->reqs.erase(it);
  return st;
}

int tlrqmc_server_stats(tlrqmc_server *s, tlrqmc_server_info *out) {
  clear_error();
  if (!s || !out) return fail(TLRQMC_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(s->mu);
  std::memset(out, 0, sizeof *out);
  out->budget_bytes = static_cast<int64_t>(s->budget);
  out->reserved_bytes = s->reserved;
  out->peak_reserved_bytes = s->peak_reserved;
  out->arena_in_use_bytes = static_cast<int64_t>(s->arena.in_use());
  out->arena_peak_bytes = static_cast<int64_t>(s->arena.peak());
  out->steps = s->steps;
  out->launches = s->launches;
  out->slot_steps = s->slot_steps;
  out->max_active_slots = s->max_active;
  out->queued = static_cast<int32_t>(s->queued.size());
  out->in_setup = s->in_setup;
  out->ready = static_cast<int32_t>(s->ready.size());
  out->running = static_cast<int32_t>(s->running.size());
  return TLRQMC_OK;
}

int tlrqmc_server_destroy(tlrqmc_server *s) {
  clear_error();
  if (!s) return TLRQMC_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    s->cv.notify_all();
  }
  for (auto &t : s->t_setup) t.join();
  s->t_run.join();
  (void)hipSetDevice(s->user->device);
  (void)hipStreamSynchronize(s->rctx.stream);
  for (auto &c : s->sctx) (void)hipStreamSynchronize(c.stream);
  for (auto &kv : s->reqs) s->release(kv.second.get());
  for (int k = 0; k < 2; ++k) {
    if (s->h_desc[k]) (void)hipHostFree(s->h_desc[k]);
    if (s->ev[k]) (void)hipEventDestroy(s->ev[k]);
  }
  std::vector<tlrqmc_ctx *> all{&s->rctx};
  for (auto &c : s->sctx) all.push_back(&c);
  for (tlrqmc_ctx *c : all) {
    (void)hipStreamDestroy(c->stream);
    c->release_pinned();
    release_blas(c);
  }
  s->arena.release(s->user);
  delete s;
  return TLRQMC_OK;
}

}  // extern "C"

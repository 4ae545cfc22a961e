// Internal declarations of libtlrqmc: context, factor, kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "plan.hpp"
#include "tlrqmc.h"

namespace tlrqmc {

// Thread-local error message; returns `code` for chaining.
int fail(int code, const char *fmt, ...);
void clear_error();

// Estimate from per-shift partial sums (max, sum of exp(log P - max), count
// of empty samples), as the device reduction writes them.
void estimate_from_parts(const std::vector<double> &part, int M, int64_t N, tlrqmc_result *out);


// Device buffers of one call, released on scope exit (through the context's
// allocator).
struct Scratch {
  tlrqmc_ctx *ctx;
  std::vector<void *> ptrs;
  explicit Scratch(tlrqmc_ctx *c) : ctx(c) {}
  ~Scratch();
  template <class T>
  T *get(size_t count);
};

// Events created during one call, destroyed on scope exit.
struct Events {
  std::vector<hipEvent_t> evs;
  ~Events() {
    for (hipEvent_t e : evs) (void)hipEventDestroy(e);
  }
  hipEvent_t make() {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    evs.push_back(e);
    return e;
  }
};

}  // namespace tlrqmc

struct tlrqmc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  tlrqmc_allocator alloc{};
  bool has_alloc = false;
  // Worker streams (default priority) on which independent sample chunks
  // run concurrently, so that the last partial round of waves of one
  // chunk's launch is filled by another chunk's work.
  std::vector<hipStream_t> workers;
  // Pinned host staging buffers (factor download), kept between calls.
  std::vector<std::pair<void *, size_t>> staging;
  // Timing events of profiled calls, kept between calls (a profiled call
  // takes two per launch).
  std::vector<hipEvent_t> event_pool;
  void *blas = nullptr;  // rocblas_handle, created by the first factor build
  void *dmalloc(size_t bytes);
  void dfree(void *p);
  int worker_streams(int count);
  double *pinned(int slot, size_t bytes);
  void release_pinned();
};


namespace tlrqmc {

// The context stream is drained before the buffers go back: after the
// synchronizations of the normal paths this costs nothing, and on an error
// path it keeps a buffer from reaching its next user while a kernel queued
// before the error still uses it.
inline Scratch::~Scratch() {
  if (!ptrs.empty()) (void)hipStreamSynchronize(ctx->stream);
  for (void *p : ptrs) ctx->dfree(p);
}

template <class T>
T *Scratch::get(size_t count) {
  if (count == 0) count = 1;
  void *p = ctx->dmalloc(count * sizeof(T));
  if (p) ptrs.push_back(p);
  return static_cast<T *>(p);
}

// Destroy a context's cached rocBLAS handle (setup.cpp).
void release_blas(tlrqmc_ctx *ctx);

// ---- device lock (setup.cpp) ----
// rocSOLVER / rocBLAS factorizations returned wrong factors (errors of 0.1 in
// entries of L, starting a few panels in) while this library's estimator
// kernels ran beside them on other streams; on an idle device, or beside
// other kernels that were tried, they are exact and reproducible.  So every
// library factorization call runs with the device to itself: it holds this
// lock exclusively, after draining the device, and every section of this
// library that launches its own kernels holds it shared.  Writers are
// preferred, so short shared sections cannot starve a factorization.  Shared
// holds nest within a thread; an exclusive section entered while the thread
// holds it shared gives that hold up for its duration (the drain completes
// the thread's own work first).
class DeviceLock {
 public:
  void lock_shared();
  void unlock_shared();
  void lock();
  void unlock();

 private:
  std::mutex mu_;
  std::condition_variable cv_;
  int readers_ = 0, writers_waiting_ = 0;
  bool writer_ = false;
};
DeviceLock &device_lock();

// Scope holding the device lock shared (kernel launches of this library).
class SharedDevice {
 public:
  SharedDevice();
  ~SharedDevice();
  SharedDevice(const SharedDevice &) = delete;
  SharedDevice &operator=(const SharedDevice &) = delete;
};

// Scope holding the device lock exclusively with the device drained; `ok`
// is false when the drain failed.  The scope's library calls must be
// complete (their stream synchronized) before it ends.
class ExclusiveDevice {
 public:
  ExclusiveDevice();
  ~ExclusiveDevice();
  ExclusiveDevice(const ExclusiveDevice &) = delete;
  ExclusiveDevice &operator=(const ExclusiveDevice &) = delete;
  bool ok = false;

 private:
  int held_shared_ = 0;
};


// ---- dense device linear algebra shared by the clients (setup.cpp) ----
// The context's rocBLAS handle on its stream (rocblas_handle).
typedef struct _rocblas_handle *rocblas_handle_t;
rocblas_handle_t blas_handle(tlrqmc_ctx *ctx);
// Cholesky (lower) of the n x n device matrix A in place; ENOTSPD names the column.
int device_cholesky(tlrqmc_ctx *ctx, double *A, int64_t lda, int64_t n);
// TLR factor of the symmetric device matrix S (lower stored, leading
// dimension lds): geometric order of xy (identity when xy is null), then
// the Cholesky (order 0) or the block reordering during the Cholesky with
// limits a, b (order 2), then the tile compression of tlr_factor.
int factor_from_device_dense(tlrqmc_ctx *ctx, int64_t n, const double *S, int64_t lds, const double *a,
                             const double *b, const double *xy, int m, double tol, int max_rank, int order,
                             int32_t *perm_out, tlrqmc_factor **out);

// ---- no-allocation scratch (noalloc.hip) ----
// Size of the file-scope device array behind tlrqmc_prob_noalloc.
int64_t noalloc_scratch_bytes();
// Resolve (once per device, with the device made current) and keep the
// array's device address; TLRQMC_EDEVICE with a message on failure.
int noalloc_resolve(int device);
// The array's address on `device`, or null if it was not resolved.
void *noalloc_scratch(int device);

// ---- host lattice (lattice.cpp) ----
std::vector<uint64_t> richtmyer_generators(int64_t dim);
std::vector<uint64_t> splitmix64_table(uint64_t seed, int64_t count);

// ---- factor construction (factor.cpp) ----
int factor_build(tlrqmc_ctx *ctx, int64_t n, int m, const int32_t *perm, const double *diag,
                 const int32_t *ranks, const double *U, const double *V, int cap_hits,
                 tlrqmc_factor **out);

// ---- kernels (kernels.hip, kernels_lr64.hip, kernels_mfma.hip) ----
// Optional start and stop events of one launch: when given, the launch
// itself marks them (hipExtLaunchKernel), with no separate marker packets
// in the stream.
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};
void launch_lr_mfma(hipStream_t s, const MfmaLrParams &p, const LaunchEvents &ev = {});
void launch_init(hipStream_t s, const InitParams &p, const LaunchEvents &ev = {});
void launch_sweep(hipStream_t s, const SweepParams &p, bool two_sided, bool scaled, bool prec,
                  const LaunchEvents &ev = {});
void launch_delta_f64(hipStream_t s, const LrParams &p, const LaunchEvents &ev = {});
void launch_zproj_f64(hipStream_t s, const LrParams &p, const LaunchEvents &ev = {});
void launch_reduce(hipStream_t s, const ReduceParams &p, int n_shifts, const LaunchEvents &ev = {});

// Batched launches: d points to n descriptors in device memory; slot i's
// launch is the one its descriptor would make alone.
void launch_init_batch(hipStream_t s, const InitParams *d, int n, int64_t max_count);
void launch_sweep_batch(hipStream_t s, const SweepParams *d, int n, int64_t max_count, bool two_sided, bool scaled,
                        bool prec);
void launch_delta_f64_batch(hipStream_t s, const LrParams *d, int n, int64_t max_count, int max_rows);
void launch_zproj_f64_batch(hipStream_t s, const LrParams *d, int n, int64_t max_count, int max_rows);
void launch_reduce_batch(hipStream_t s, const ReduceParams *d, int n, int max_shifts);
void launch_lr_mfma_batch(hipStream_t s, const MfmaLrParams *d, int n, int rt, bool fp64_b, bool map,
                          int64_t max_blocks);

}  // namespace tlrqmc

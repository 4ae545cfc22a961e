// Issue probe for the roofline model of bench.py: does a matrix-core wave
// hold back a vector wave on the same SIMD?
//
// One work-group of 512 threads per CU: waves 0-3 (one per SIMD) run a
// chain of matrix-core instructions (or nothing, or FP64 vector FMAs),
// waves 4-7 (again one per SIMD) run four independent chains of FMAs.
// Each wave records its own cycle count (s_memtime); the program prints
// the means.  A vector wave that takes about as long beside the matrix
// wave as alone runs beside it; one that takes the sum of both times is
// held back by it.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

constexpr int kIters = 2048;   // FMAs per chain of a vector wave
constexpr int kBlocks = 256;   // one work-group per CU
constexpr int kThreads = 512;  // eight waves: two per SIMD

// MODE: 0 nothing, 1 FP64 16x16x4 MFMA, 2 BF16 16x16x32 MFMA, 3 FP64 vector
// FMAs, 4 INT8 16x16x64 MFMA (kIters / 4 matrix instructions per chain,
// four chains).
// V64: the vector waves run FP64 (true) or FP32 (false) FMAs.
template <int MODE, bool V64>
__global__ __launch_bounds__(kThreads) void k_probe(float a, double ad, float *out, long long *cyc) {
  const int w = static_cast<int>(threadIdx.x) >> 6;
  const int t = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
  const long long t0 = clock64();
  float r = 0.f;
  if (w < 4) {
    if constexpr (MODE == 1) {
      f64x4 c[4] = {};
      const double x = t * 1e-9, y = 1e-9;
      for (int it = 0; it < kIters / 4; ++it)
#pragma unroll
        for (int m = 0; m < 4; ++m) c[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c[m], 0, 0, 0);
      r = static_cast<float>(c[0][0] + c[1][1] + c[2][2] + c[3][3]);
    } else if constexpr (MODE == 2) {
      f32x4 c[4] = {};
      bf16x8 x = {}, y = {};
      x[0] = static_cast<__bf16>(t * 1e-9f);
      for (int it = 0; it < kIters / 4; ++it)
#pragma unroll
        for (int m = 0; m < 4; ++m) c[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, c[m], 0, 0, 0);
      r = c[0][0] + c[1][1] + c[2][2] + c[3][3];
    } else if constexpr (MODE == 4) {
      i32x4 c[4] = {};
      i32x4 x = {t, 1, 2, 3}, y = {3, 2, 1, t};
      for (int it = 0; it < kIters / 4; ++it)
#pragma unroll
        for (int m = 0; m < 4; ++m) c[m] = __builtin_amdgcn_mfma_i32_16x16x64_i8(x, y, c[m], 0, 0, 0);
      r = static_cast<float>(c[0][0] + c[1][1] + c[2][2] + c[3][3]);
    } else if constexpr (MODE == 3) {
      double x0 = t * 1e-9, x1 = x0 + 1, x2 = x0 + 2, x3 = x0 + 3;
      for (int it = 0; it < kIters; ++it) {
        x0 = fma(x0, ad, 1e-7);
        x1 = fma(x1, ad, 1e-7);
        x2 = fma(x2, ad, 1e-7);
        x3 = fma(x3, ad, 1e-7);
      }
      r = static_cast<float>(x0 + x1 + x2 + x3);
    }
  } else if constexpr (V64) {
    double x0 = t * 1e-9, x1 = x0 + 1, x2 = x0 + 2, x3 = x0 + 3;
    for (int it = 0; it < kIters; ++it) {
      x0 = fma(x0, ad, 1e-7);
      x1 = fma(x1, ad, 1e-7);
      x2 = fma(x2, ad, 1e-7);
      x3 = fma(x3, ad, 1e-7);
    }
    r = static_cast<float>(x0 + x1 + x2 + x3);
  } else {
    float x0 = t * 1e-9f, x1 = x0 + 1, x2 = x0 + 2, x3 = x0 + 3;
    for (int it = 0; it < kIters; ++it) {
      x0 = fmaf(x0, a, 1e-7f);
      x1 = fmaf(x1, a, 1e-7f);
      x2 = fmaf(x2, a, 1e-7f);
      x3 = fmaf(x3, a, 1e-7f);
    }
    r = x0 + x1 + x2 + x3;
  }
  const long long t1 = clock64();
  out[t] = r;
  if ((threadIdx.x & 63) == 0) cyc[t / 64] = t1 - t0;
}

void check(hipError_t e, const char *what) {
  if (e != hipSuccess) {
    std::fprintf(stderr, "issue_probe: %s: %s\n", what, hipGetErrorString(e));
    std::exit(1);
  }
}

template <int MODE, bool V64>
void run(const char *name, float *out, long long *cyc) {
  for (int rep = 0; rep < 2; ++rep) {  // the second launch is the one read
    hipLaunchKernelGGL((k_probe<MODE, V64>), dim3(kBlocks), dim3(kThreads), 0, 0, 1.0000001f, 1.0000001, out, cyc);
    check(hipGetLastError(), "launch");
    check(hipDeviceSynchronize(), "synchronize");
  }
  std::vector<long long> h(kBlocks * 8);
  check(hipMemcpy(h.data(), cyc, h.size() * sizeof(long long), hipMemcpyDeviceToHost), "copy");
  double a = 0, b = 0;
  for (int i = 0; i < kBlocks; ++i)
    for (int w = 0; w < 8; ++w) (w < 4 ? a : b) += static_cast<double>(h[i * 8 + w]);
  a /= kBlocks * 4;
  b /= kBlocks * 4;
  std::printf("| %s | %.0f | %s | %.0f | %.2f |\n", name, a, V64 ? "FP64" : "FP32", b, b / (4.0 * kIters));
}

}  // namespace

int main() {
  float *out = nullptr;
  long long *cyc = nullptr;
  check(hipMalloc(&out, kBlocks * kThreads * sizeof(float)), "alloc");
  check(hipMalloc(&cyc, kBlocks * 8 * sizeof(long long)), "alloc");
  std::printf("| waves 0-3 | their cycles | waves 4-7 (4 x %d FMAs) | their cycles | cycles per FMA instruction |\n",
              kIters);
  std::printf("|---|---:|---|---:|---:|\n");
  run<0, false>("nothing", out, cyc);
  run<1, false>("512 x 4 FP64 16x16x4 MFMA", out, cyc);
  run<2, false>("512 x 4 BF16 16x16x32 MFMA", out, cyc);
  run<3, false>("4 x 2048 FP64 vector FMAs", out, cyc);
  run<4, false>("512 x 4 INT8 16x16x64 MFMA", out, cyc);
  run<0, true>("nothing", out, cyc);
  run<1, true>("512 x 4 FP64 16x16x4 MFMA", out, cyc);
  run<2, true>("512 x 4 BF16 16x16x32 MFMA", out, cyc);
  run<3, true>("4 x 2048 FP64 vector FMAs", out, cyc);
  run<4, true>("512 x 4 INT8 16x16x64 MFMA", out, cyc);
  check(hipFree(out), "free");
  check(hipFree(cyc), "free");
  return 0;
}

// Issue-rate microbenchmark behind the image kernel's instruction roofline:
// wave64 VALU instructions per CU per clock for independent FP32 FMA chains,
// against the number of waves per SIMD (set by the dynamic LDS each
// workgroup reserves), for three instruction mixes:
//   fma1  a = fma(a, 0.999, 1e-4)            one VGPR operand
//   fma3  a = fma(a, c, d)                   three VGPR operands
//   fmas  a = fma(a, s, d)                   two VGPR operands and one SGPR
//   sin   8 fma3 + 2 v_sin_f32 per 8 chains  cost of a transcendental
// Clock and CU count are the MI355X's (2.4 GHz, 256 CUs). Standalone
// program; built next to the library by the package's build script.
#include <hip/hip_runtime.h>

#include <cstdio>

#define CHECK(x)                                                                           \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) {                                                                \
      std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);           \
      return 1;                                                                            \
    }                                                                                      \
  } while (0)

constexpr int kChains = 8;
constexpr int kThreads = 256;
constexpr int kBlocks = 256 * 16;
constexpr int kIters = 1024;

template <int MIX>
__global__ __launch_bounds__(kThreads) void chains(float* out, int iters, float su) {
  extern __shared__ float reserve[];   // occupancy control only
  float a[kChains], c[kChains];
  for (int i = 0; i < kChains; ++i) {
    a[i] = 0.3f + threadIdx.x * 1e-3f + i * 0.1f;
    c[i] = 0.999f + threadIdx.x * 1e-7f * i;
  }
  const float d = 1e-4f * threadIdx.x;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kChains; ++i) {
      if (MIX == 0) {
        a[i] = __builtin_fmaf(a[i], 0.999f, 1e-4f);
      } else if (MIX == 3) {
        a[i] = __builtin_fmaf(a[i], su, c[i]);
      } else {
        a[i] = __builtin_fmaf(a[i], c[i], d);
        if (MIX == 2 && (i & 3) == 0) a[i] = __builtin_amdgcn_sinf(a[i]);
      }
    }
  }
  float s = 0.0f;
  for (int i = 0; i < kChains; ++i) s += a[i];
  if (threadIdx.x == 0) reserve[0] = s;
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <int MIX>
int run(const char* name, float* out, int lds) {
  CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(chains<MIX>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds));
  int per_cu = 0;
  CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, chains<MIX>, kThreads, lds));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  hipLaunchKernelGGL(chains<MIX>, dim3(kBlocks), dim3(kThreads), lds, 0, out, kIters, 0.999f);   // warm-up
  CHECK(hipGetLastError());
  CHECK(hipEventRecord(e0));
  hipLaunchKernelGGL(chains<MIX>, dim3(kBlocks), dim3(kThreads), lds, 0, out, kIters, 0.999f);
  CHECK(hipGetLastError());
  CHECK(hipEventRecord(e1));
  CHECK(hipEventSynchronize(e1));
  float ms = 0.0f;
  CHECK(hipEventElapsedTime(&ms, e0, e1));
  const double per_iter = kChains + (MIX == 2 ? 2.0 : 0.0);
  const double waves = (double)kBlocks * kThreads / 64.0;
  const double rate = waves * kIters * per_iter / (ms * 1e-3 * 2.4e9 * 256.0);
  // a 256-thread workgroup puts one wave on each of the four SIMDs of a CU
  std::printf("%-5s waves/SIMD %d  %.3f ms  %.3f wave-instructions per CU per clock\n", name, per_cu, ms, rate);
  CHECK(hipEventDestroy(e0));
  CHECK(hipEventDestroy(e1));
  return 0;
}

int main() {
  float* out = nullptr;
  CHECK(hipMalloc(&out, sizeof(float) * kBlocks * kThreads));
  const int lds[] = {150 * 1024, 76 * 1024, 50 * 1024, 38 * 1024, 30 * 1024, 18 * 1024};
  for (int l : lds)
    if (run<0>("fma1", out, l)) return 1;
  for (int l : lds)
    if (run<1>("fma3", out, l)) return 1;
  for (int l : lds)
    if (run<3>("fmas", out, l)) return 1;
  for (int l : lds)
    if (run<2>("sin", out, l)) return 1;
  CHECK(hipFree(out));
  return 0;
}

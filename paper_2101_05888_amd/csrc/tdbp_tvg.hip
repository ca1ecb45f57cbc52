// Time-varying gain of an echo cube (Eq. 10, Sec. II-E).
//
// For each sample time t the population median power over every (ping,
// element) of the cube, P~(t) (the element of rank floor((N - 1) / 2) of the
// N = P E values |E[p, e, t]|^2), and G(t) = (alpha mean_t P~ + P~(t))^-1, a
// power gain applied to the complex samples as sqrt(G(t)) (samples of a time
// whose gain is not finite are left unchanged).
//
// The medians are exact radix selections on the FP32 bit patterns of |E|^2
// (non-negative values order like their bits): a workgroup owns 16
// consecutive sample times, reads its 16-sample run of every (ping, element)
// row (one 128-byte line per row), and per pass of 11, 11 and 10 bits builds
// one LDS histogram per sample time of the keys that share the digits found
// so far; 16 threads per sample time then find the digit holding the rank.
// With at most 65535 rows two 16-bit counts share each 32-bit LDS word (no
// count can carry into its neighbour), halving the histograms to 64 KB so
// that two workgroups fit a CU. The mean over sample times is a fixed-order
// FP64 sum.
#include "tdbp_dev.h"

namespace sasbp {

constexpr int kTvgCols = 16;     // sample times per workgroup
constexpr int kTvgBins = 2048;

__device__ __forceinline__ unsigned tvg_key(float2 v) { return __float_as_uint(fmaf(v.x, v.x, v.y * v.y)); }

template <bool PACK>
__global__ __launch_bounds__(kThreads) void tvg_median_kernel(const float2* echo, long long rows, int Ns,
                                                              float* med) {
  constexpr int WORDS = PACK ? kTvgBins / 2 : kTvgBins;
  __shared__ unsigned hist[kTvgCols][WORDS];
  auto count = [&](int c, int d) -> unsigned {
    return PACK ? (hist[c][d >> 1] >> ((d & 1) << 4)) & 0xFFFFu : hist[c][d];
  };
  __shared__ unsigned part[kTvgCols][kThreads / kTvgCols];
  __shared__ unsigned s_prefix[kTvgCols], s_rank[kTvgCols];
  constexpr int RL = kThreads / kTvgCols;   // threads per sample time (16)
  const int tid = threadIdx.x;
  const int col = tid % kTvgCols, lane = tid / kTvgCols;
  const int t0 = blockIdx.x * kTvgCols;
  const bool valid = t0 + col < Ns;
  if (tid < kTvgCols) {
    s_prefix[tid] = 0u;
    s_rank[tid] = (unsigned)((rows - 1) / 2);
  }
  for (int pass = 0; pass < 3; ++pass) {
    for (int i = tid; i < kTvgCols * WORDS; i += kThreads) (&hist[0][0])[i] = 0u;
    __syncthreads();
    const int shift = pass == 0 ? 21 : (pass == 1 ? 10 : 0);
    const unsigned mask = pass == 2 ? 0x3FFu : 0x7FFu;
    const unsigned prefix = s_prefix[col];
    if (valid) {
      for (long long r = lane; r < rows; r += RL) {
        const unsigned key = tvg_key(echo[r * Ns + t0 + col]);
        const bool match = pass == 0 || (key >> (shift + (pass == 1 ? 11 : 10))) == prefix;
        const unsigned b = (key >> shift) & mask;
        if (match) {
          if (PACK) atomicAdd(&hist[col][b >> 1], 1u << ((b & 1u) << 4));
          else atomicAdd(&hist[col][b], 1u);
        }
      }
    }
    __syncthreads();
    // digit selection: the 16 threads of a sample time each sum 128 bins
    constexpr int PER = kTvgBins / RL;
    const int bins = pass == 2 ? 1024 : 2048;
    unsigned sum = 0u;
    for (int j = 0; j < PER; ++j) {
      const int d = lane * PER + j;
      sum += d < bins ? count(col, d) : 0u;
    }
    part[col][lane] = sum;
    __syncthreads();
    unsigned before = 0u;
    for (int l = 0; l < lane; ++l) before += part[col][l];
    const unsigned k = s_rank[col];
    __syncthreads();
    if (valid && k >= before && k < before + sum) {   // exactly one thread per sample time
      unsigned r = k - before;
      int d = lane * PER;
      for (int j = 0; j < PER; ++j) {
        const unsigned c = count(col, lane * PER + j);
        if (r < c) { d = lane * PER + j; break; }
        r -= c;
      }
      s_rank[col] = r;
      s_prefix[col] = (s_prefix[col] << (pass == 2 ? 10 : 11)) | (unsigned)d;
    }
    __syncthreads();
  }
  if (lane == 0 && valid) med[t0 + col] = __uint_as_float(s_prefix[col]);
}

// mean of the medians (fixed-order FP64) and the amplitude factor per time
__global__ __launch_bounds__(kThreads) void tvg_gain_kernel(const float* med, int Ns, double alpha, float* amp,
                                                            float* gain_out) {
  __shared__ double part[kThreads];
  double s = 0.0;
  for (int t = threadIdx.x; t < Ns; t += kThreads) s += (double)med[t];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  const double mean = part[0] / (double)Ns;
  for (int t = threadIdx.x; t < Ns; t += kThreads) {
    const double G = 1.0 / (alpha * mean + (double)med[t]);
    amp[t] = isfinite(G) ? (float)sqrt(G) : 1.0f;
    if (gain_out) gain_out[t] = (float)G;
  }
}

__global__ __launch_bounds__(kThreads) void tvg_apply_kernel(float2* echo, long long n, int Ns, const float* amp) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float a = amp[i % Ns];
    const float2 v = echo[i];
    echo[i] = make_float2(v.x * a, v.y * a);
  }
}

hipError_t launch_tvg(void* echo, long long rows, int Ns, double alpha, float* work, float* gain_out,
                      hipStream_t st) {
  float2* e = reinterpret_cast<float2*>(echo);
  float* med = work;
  float* amp = work + Ns;
  const int groups = (Ns + kTvgCols - 1) / kTvgCols;
  if (rows <= 65535)
    hipLaunchKernelGGL(tvg_median_kernel<true>, dim3(groups), dim3(kThreads), 0, st, (const float2*)e, rows, Ns, med);
  else
    hipLaunchKernelGGL(tvg_median_kernel<false>, dim3(groups), dim3(kThreads), 0, st, (const float2*)e, rows, Ns,
                       med);
  hipLaunchKernelGGL(tvg_gain_kernel, dim3(1), dim3(kThreads), 0, st, (const float*)med, Ns, alpha, amp, gain_out);
  const long long n = rows * (long long)Ns;
  long long blocks = (n + kThreads - 1) / kThreads;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(tvg_apply_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, st, e, n, Ns, (const float*)amp);
  return hipGetLastError();
}

}  // namespace sasbp

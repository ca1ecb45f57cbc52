// Dynamic range compression of an image for display (Eqs. 11-12, Sec. II-E).
//
// The input is the magnitude of the complex image normalised by its maximum,
// x = |I| / max |I|. Each pixel maps to q x / ((q - 1) x + 1), with q chosen so
// that the median pixel maps to the requested brightness b:
// q = (b - b x~) / (x~ - b x~), x~ the median of x (the element of rank
// floor((N - 1) / 2) in ascending order). Degenerate images: all zero -> all
// zero (q = 1); x~ = 0 -> every non-zero pixel to 1 (q = inf); x~ = 1 ->
// every pixel below the maximum to 0 (q = 0).
//
// Squared magnitudes order like magnitudes, and non-negative FP32 values
// order like their bit patterns, so the maximum is an integer atomic max and
// the median an exact radix select on the 32-bit keys of |I|^2: three passes
// of 11, 11 and 10 bits, each a histogram (LDS, then global integer atomics)
// of the keys that share the digits found so far, then a one-workgroup scan
// that picks the digit holding the wanted rank.
#include "tdbp_dev.h"

namespace sasbp {

constexpr int kDrcBins = 2048;

// hdr: [0] max key, [1] rank still wanted, [2] key prefix found so far
struct DrcWork {
  unsigned hdr[16];
  unsigned hist[kDrcBins];
  double params[4];   // max |I|, median of x, q
};

__device__ __forceinline__ unsigned drc_key(float2 v) { return __float_as_uint(fmaf(v.x, v.x, v.y * v.y)); }

__global__ __launch_bounds__(kThreads) void drc_init_kernel(DrcWork* w, long long n) {
  for (int i = threadIdx.x; i < kDrcBins; i += blockDim.x) w->hist[i] = 0u;
  if (threadIdx.x == 0) {
    w->hdr[0] = 0u;
    w->hdr[1] = (unsigned)((n - 1) / 2);
    w->hdr[2] = 0u;
  }
}

__global__ __launch_bounds__(kThreads) void drc_max_kernel(const float2* img, long long n, DrcWork* w) {
  unsigned m = 0u;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    m = max(m, drc_key(img[i]));
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(&w->hdr[0], m);
}

// pass 0: digit = key[31:21]; pass 1: key[20:10] of keys with key[31:21] ==
// prefix; pass 2: key[9:0] of keys with key[31:10] == prefix
__global__ __launch_bounds__(kThreads) void drc_hist_kernel(const float2* img, long long n, DrcWork* w, int pass) {
  __shared__ unsigned h[kDrcBins];
  for (int i = threadIdx.x; i < kDrcBins; i += blockDim.x) h[i] = 0u;
  __syncthreads();
  const unsigned prefix = w->hdr[2];
  const int shift = pass == 0 ? 21 : (pass == 1 ? 10 : 0);
  const unsigned mask = pass == 2 ? 0x3FFu : 0x7FFu;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const unsigned key = drc_key(img[i]);
    const bool match = pass == 0 || (key >> (shift + (pass == 1 ? 11 : 10))) == prefix;
    if (match) atomicAdd(&h[(key >> shift) & mask], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kDrcBins; i += blockDim.x)
    if (h[i]) atomicAdd(&w->hist[i], h[i]);
}

// Find the digit holding the wanted rank: each of the 256 threads sums 8
// bins, an inclusive scan over the threads gives each group's start, and the
// thread whose group holds the rank walks its 8 bins.
__global__ __launch_bounds__(kThreads) void drc_select_kernel(DrcWork* w, int pass, double b, double* params_out) {
  constexpr int PER = kDrcBins / kThreads;   // 8 bins per thread
  __shared__ unsigned scan[kThreads];
  const int t = threadIdx.x;
  const int bins = pass == 2 ? 1024 : 2048;
  unsigned c[PER];
  unsigned sum = 0u;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int d = t * PER + j;
    c[j] = d < bins ? w->hist[d] : 0u;
    sum += c[j];
  }
  scan[t] = sum;
  __syncthreads();
  for (int o = 1; o < kThreads; o <<= 1) {   // inclusive scan
    const unsigned v = t >= o ? scan[t - o] : 0u;
    __syncthreads();
    scan[t] += v;
    __syncthreads();
  }
  const unsigned k = w->hdr[1];
  const unsigned before = t > 0 ? scan[t - 1] : 0u;
  __syncthreads();
  if (k >= before && k < scan[t]) {   // exactly one thread: this group holds rank k
    unsigned r = k - before;
    int d = t * PER;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      if (r < c[j]) { d = t * PER + j; break; }
      r -= c[j];
    }
    w->hdr[1] = r;
    w->hdr[2] = (w->hdr[2] << (pass == 2 ? 10 : 11)) | (unsigned)d;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kDrcBins; i += blockDim.x) w->hist[i] = 0u;
  if (pass == 2 && threadIdx.x == 0) {
    const double peak = sqrt((double)__uint_as_float(w->hdr[0]));
    double med = 0.0, q = 1.0;
    if (peak > 0.0) {
      med = sqrt((double)__uint_as_float(w->hdr[2])) / peak;
      if (med <= 0.0) q = __longlong_as_double(0x7ff0000000000000ll);   // +inf
      else if (med >= 1.0) q = 0.0;
      else q = (b - b * med) / (med - b * med);
    }
    w->params[0] = peak;
    w->params[1] = med;
    w->params[2] = q;
    if (params_out) {
      params_out[0] = peak;
      params_out[1] = med;
      params_out[2] = q;
    }
  }
}

__global__ __launch_bounds__(kThreads) void drc_map_kernel(const float2* img, long long n, const DrcWork* w,
                                                           float* out) {
  const float peak = (float)w->params[0];
  const double qd = w->params[2];
  const float inv = peak > 0.0f ? 1.0f / peak : 0.0f;
  const float q = (float)qd;
  const bool qinf = isinf(qd), qzero = qd == 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float2 v = img[i];
    const float x = fminf(sqrtf(fmaf(v.x, v.x, v.y * v.y)) * inv, 1.0f);
    float y;
    if (!(peak > 0.0f)) y = 0.0f;
    else if (qinf) y = x > 0.0f ? 1.0f : 0.0f;
    else if (qzero) y = x >= 1.0f ? 1.0f : 0.0f;
    else y = q * x / fmaf(q - 1.0f, x, 1.0f);
    out[i] = y;
  }
}

hipError_t launch_drc(const void* image, long long n, double brightness, float* out, double* params, void* work,
                      hipStream_t st) {
  const float2* img = reinterpret_cast<const float2*>(image);
  DrcWork* w = reinterpret_cast<DrcWork*>(work);
  long long blocks = (n + kThreads - 1) / kThreads;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(drc_init_kernel, dim3(1), dim3(kThreads), 0, st, w, n);
  hipLaunchKernelGGL(drc_max_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, st, img, n, w);
  for (int pass = 0; pass < 3; ++pass) {
    hipLaunchKernelGGL(drc_hist_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, st, img, n, w, pass);
    hipLaunchKernelGGL(drc_select_kernel, dim3(1), dim3(kThreads), 0, st, w, pass, brightness, params);
  }
  hipLaunchKernelGGL(drc_map_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, st, img, n, w, out);
  return hipGetLastError();
}

size_t drc_work_bytes() { return sizeof(DrcWork); }

}  // namespace sasbp

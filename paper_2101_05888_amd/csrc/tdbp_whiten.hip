// Spectral whitening of an echo cube (Eq. 9, Sec. II-E).
//
// Every (ping, element) row of N_s samples is transformed (batched complex
// FFT, rocFFT through hipFFT, in place). The power estimate of bin f is the
// average over rows of |X(f)|^2, summed in FP64 in a fixed order (partial
// sums over 64 row blocks, then the blocks in order); with its mean over
// bins, G(f) = 1 / (gamma mean P^ + P^(f)), normalised to max G = 1 (0 dB
// smallest attenuation), is a power gain: every spectrum is multiplied by
// sqrt(G(f)) / N_s (the inverse transform's scale folded in) and transformed
// back.
#include <hipfft/hipfft.h>

#include "tdbp_dev.h"

namespace sasbp {

constexpr int kWhitenBlocks = 64;   // row blocks of the partial power sums

__global__ __launch_bounds__(kThreads) void whiten_power_kernel(const float2* X, long long rows, int Ns,
                                                                double* part) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (f >= Ns) return;
  const long long r0 = rows * b / kWhitenBlocks, r1 = rows * (b + 1) / kWhitenBlocks;
  double s = 0.0;
  for (long long r = r0; r < r1; ++r) {
    const float2 v = X[r * Ns + f];
    s += (double)v.x * v.x + (double)v.y * v.y;
  }
  part[(size_t)b * Ns + f] = s;
}

__global__ __launch_bounds__(kThreads) void whiten_gain_kernel(const double* part, long long rows, int Ns,
                                                               double gamma, double* phat, float* amp) {
  __shared__ double red[kThreads];
  // P^(f) in fixed block order, and the sum over bins
  double tot = 0.0;
  for (int f = threadIdx.x; f < Ns; f += kThreads) {
    double s = 0.0;
    for (int b = 0; b < kWhitenBlocks; ++b) s += part[(size_t)b * Ns + f];
    s /= (double)rows;
    phat[f] = s;
    tot += s;
  }
  red[threadIdx.x] = tot;
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  const double mean = red[0] / (double)Ns;
  __syncthreads();
  // max G = 1 / min over bins of (gamma mean + P^)
  double mn = 1.0e308;
  for (int f = threadIdx.x; f < Ns; f += kThreads) mn = fmin(mn, gamma * mean + phat[f]);
  red[threadIdx.x] = mn;
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  const double dmin = red[0];
  for (int f = threadIdx.x; f < Ns; f += kThreads) {
    const double d = gamma * mean + phat[f];
    const double g = d > 0.0 ? dmin / d : 1.0;   // G / max G
    amp[f] = (float)(sqrt(g) / (double)Ns);
  }
}

__global__ __launch_bounds__(kThreads) void whiten_apply_kernel(float2* X, long long n, int Ns, const float* amp) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float a = amp[i % Ns];
    const float2 v = X[i];
    X[i] = make_float2(v.x * a, v.y * a);
  }
}

// work: kWhitenBlocks * Ns + Ns doubles, then Ns floats
size_t whiten_work_bytes(int Ns) {
  return sizeof(double) * ((size_t)kWhitenBlocks * Ns + Ns) + sizeof(float) * (size_t)Ns;
}

int launch_whiten(void* fft_plan, void* echo, long long rows, int Ns, double gamma, void* work, hipStream_t st) {
  hipfftHandle h = reinterpret_cast<hipfftHandle>(fft_plan);
  hipfftComplex* X = reinterpret_cast<hipfftComplex*>(echo);
  double* part = reinterpret_cast<double*>(work);
  double* phat = part + (size_t)kWhitenBlocks * Ns;
  float* amp = reinterpret_cast<float*>(phat + Ns);
  if (hipfftSetStream(h, st) != HIPFFT_SUCCESS) return 1;
  if (hipfftExecC2C(h, X, X, HIPFFT_FORWARD) != HIPFFT_SUCCESS) return 2;
  hipLaunchKernelGGL(whiten_power_kernel, dim3((Ns + kThreads - 1) / kThreads, kWhitenBlocks), dim3(kThreads), 0, st,
                     (const float2*)echo, rows, Ns, part);
  hipLaunchKernelGGL(whiten_gain_kernel, dim3(1), dim3(kThreads), 0, st, (const double*)part, rows, Ns, gamma, phat,
                     amp);
  const long long n = rows * (long long)Ns;
  long long blocks = (n + kThreads - 1) / kThreads;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(whiten_apply_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, st, (float2*)echo, n, Ns,
                     (const float*)amp);
  if (hipGetLastError() != hipSuccess) return 3;
  if (hipfftExecC2C(h, X, X, HIPFFT_BACKWARD) != HIPFFT_SUCCESS) return 2;
  return 0;
}

int make_fft_plan(int Ns, long long rows, void** out) {
  hipfftHandle h;
  if (hipfftPlan1d(&h, Ns, HIPFFT_C2C, (int)rows) != HIPFFT_SUCCESS) return 1;
  *out = reinterpret_cast<void*>(h);
  return 0;
}

void destroy_fft_plan(void* p) {
  if (p) (void)hipfftDestroy(reinterpret_cast<hipfftHandle>(p));
}

}  // namespace sasbp

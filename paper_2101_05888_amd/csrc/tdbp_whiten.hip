// Spectral whitening of an echo cube (Eq. 9, Sec. II-E).
//
// Every (ping, element) row of N_s samples is transformed; the power estimate
// of bin f is the average over rows of |X(f)|^2, summed in FP64 in a fixed
// order (partial sums over row blocks, then the blocks in order); with its
// mean over bins, G(f) = 1 / (gamma mean P^ + P^(f)), normalised to max G = 1
// (0 dB smallest attenuation), is a power gain: every spectrum is multiplied
// by sqrt(G(f)) / N_s (the inverse transform's scale folded in) and
// transformed back.
//
// Rows of N_s = 4096 R samples (R = 1, 2, 4) take a hand-written path in two
// passes over the cube. The forward kernel keeps a row in LDS: a radix-R
// pass in registers (decimation in frequency, n = n2 + 4096 n1, k = k1 +
// R k2, twiddles W_N^(n2 k1)), then R 4096-point transforms (the radix-16
// passes of tdbp_fft.h, one 256-thread group each); it writes the spectrum
// back in place grouped by k1 (slot k1 4096 + k2 holds bin k1 + R k2) and
// keeps each thread's bins' |X|^2 in FP64 registers over its workgroup's
// fixed run of rows. The inverse kernel reads a grouped spectrum, applies
// the gain, runs the same passes with conjugate twiddles and the radix-R
// pass last, and writes the row in natural order. Other lengths use rocFFT
// (through hipFFT) with separate power, gain and scaling kernels.
#include <hipfft/hipfft.h>

#include <algorithm>

#include "tdbp_dev.h"
#include "tdbp_fft.h"

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

// P^(f): the row blocks' partial sums of bin f added in block order, over the
// row count; one thread per bin.
__global__ __launch_bounds__(kThreads) void whiten_estimate_kernel(const double* part, int nblk, long long rows,
                                                                   int Ns, double* phat) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= Ns) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(size_t)b * Ns + f];
  phat[f] = s / (double)rows;
}

__global__ __launch_bounds__(kThreads) void whiten_gain_kernel(int Ns, double gamma, const double* phat, float* amp) {
  __shared__ double red[kThreads];
  // the sum of P^ over bins, in a fixed order
  double tot = 0.0;
  for (int f = threadIdx.x; f < Ns; f += kThreads) tot += phat[f];
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

// ----------------------------------------------------- hand-written path ---

constexpr size_t kWhitenPartWords = 1u << 22;   // FP64 partial sums of the hand-written path (32 MB)
constexpr int kWhitenTw = kFftTw + 3 * 4096;  // 4096-point table, then W_N^(n2 k1) for k1 = 1..3

__host__ __device__ inline int whiten_radix(int Ns) { return Ns == 4096 ? 1 : Ns == 8192 ? 2 : Ns == 16384 ? 4 : 0; }

// The twiddle tables, rounded from FP64: tdbp_fft.h's 4096-point table, then
// W_N^(n2 k1) at kFftTw + (k1 - 1) 4096 + n2 (W_N = exp(-2 pi i / N)).
__global__ __launch_bounds__(kThreads) void whiten_tables_kernel(float2* tw, int R) {
  const int N = 4096 * R, n = kFftTw + (R - 1) * 4096;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double sn, cs;
    if (i < kFftTw) {
      sincospi(-2.0 * (double)fft_tw_exponent(i) / (double)kFftN, &sn, &cs);
    } else {
      const int j = i - kFftTw;
      sincospi(-2.0 * (double)((j % 4096) * (j / 4096 + 1)) / (double)N, &sn, &cs);
    }
    tw[i] = make_float2((float)cs, (float)sn);
  }
}

// Length-R transform of u[0..R) in place (R = 2 or 4; natural order).
template <int R, bool INV>
__device__ __forceinline__ void whiten_dftR(float2* u) {
  if constexpr (R == 2) {
    const float2 a = u[0], b = u[1];
    u[0] = fft_add(a, b);
    u[1] = fft_sub(a, b);
  } else if constexpr (R == 4) {
    fft_dft4<INV>(u[0], u[1], u[2], u[3]);
  }
}

// Threads per workgroup: 256 per 4096-point group up to 512; with R = 4 each
// 256-thread half runs two of the four groups in turn (a 16384-point row
// fills 144 KB of LDS, so one workgroup per CU: 512 threads keep the
// registers of the prefetched next row without spilling).
template <int R> constexpr int whiten_threads() { return 256 * R < 512 ? 256 * R : 512; }

template <int R>
__global__ __launch_bounds__(whiten_threads<R>()) void whiten_forward_kernel(float2* X, long long rows,
                                                                            const float2* __restrict__ tw,
                                                                            double* part) {
  constexpr int N = 4096 * R, NT = whiten_threads<R>(), H = NT / 256, G = R / H, M = 4096 / NT;
  extern __shared__ __align__(16) unsigned char smem[];
  float2* L = reinterpret_cast<float2*>(smem);
  const int T = threadIdx.x, h = T >> 8, t = T & 255;
  float acc[G][16];
#pragma unroll
  for (int i = 0; i < G; ++i)
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[i][j] = 0.0f;
  const long long r0 = rows * blockIdx.x / gridDim.x, r1 = rows * (blockIdx.x + 1) / gridDim.x;
  // this thread's inputs of the first pass (n2 = T + NT m, all n1 < R), one row ahead
  float2 u[M * R];
  auto load_row = [&](long long r) {
    const float2* row = X + (size_t)r * N;
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
      for (int n1 = 0; n1 < R; ++n1) u[m * R + n1] = row[T + NT * m + 4096 * n1];
  };
  if (r0 < r1) load_row(r0);
  for (long long r = r0; r < r1; ++r) {
    float2* row = X + (size_t)r * N;
    __syncthreads();   // the previous row's last LDS reads are done
    // the radix-R pass (none for R = 1): group k1's input y_k1[n2] into LDS
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int n2 = T + NT * m;
      whiten_dftR<R, false>(u + m * R);
#pragma unroll
      for (int k1 = 1; k1 < R; ++k1) u[m * R + k1] = fft_cmul(u[m * R + k1], tw[kFftTw + (k1 - 1) * 4096 + n2]);
#pragma unroll
      for (int k1 = 0; k1 < R; ++k1) L[k1 * kFftLds + fft_lds(n2 >> 8, (n2 >> 4) & 15, n2 & 15)] = u[m * R + k1];
    }
    if (r + 1 < r1) load_row(r + 1);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < G; ++i) {
      const int g = h + H * i;
      float2* A = L + g * kFftLds;
      float2 v[16];
#pragma unroll
      for (int n1 = 0; n1 < 16; ++n1) v[n1] = A[fft_lds(n1, t >> 4, t & 15)];
      fft_pass1_compute<false>(v, t, tw);
      __syncthreads();   // every pass-1 load is done
      fft_pass1_store(v, t, A);
      __syncthreads();
      fft_pass2<false>(t, tw, A);
      __syncthreads();
      fft_pass3<false>(v, t, A);
      // this thread holds bin g + R (t + 256 j) in v[j]
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        acc[i][j] = fmaf(v[j].x, v[j].x, fmaf(v[j].y, v[j].y, acc[i][j]));
        row[g * 4096 + t + 256 * j] = v[j];
      }
    }
  }
#pragma unroll
  for (int i = 0; i < G; ++i)
#pragma unroll
    for (int j = 0; j < 16; ++j) part[(size_t)blockIdx.x * N + (h + H * i) + R * (t + 256 * j)] = (double)acc[i][j];
}

template <int R>
__global__ __launch_bounds__(whiten_threads<R>()) void whiten_inverse_kernel(float2* X, long long rows,
                                                                            const float2* __restrict__ tw,
                                                                            const float* __restrict__ amp) {
  constexpr int N = 4096 * R, NT = whiten_threads<R>(), H = NT / 256, G = R / H, M = 4096 / NT;
  extern __shared__ __align__(16) unsigned char smem[];
  float2* L = reinterpret_cast<float2*>(smem);
  const int T = threadIdx.x, h = T >> 8, t = T & 255;
  const long long r0 = rows * blockIdx.x / gridDim.x, r1 = rows * (blockIdx.x + 1) / gridDim.x;
  // this thread's gained spectrum values of group g (bins g + R (t + 256 j)),
  // one group ahead: while a group's passes run, the next group's loads (the
  // same row's next group, else the next row's first) are in flight
  float2 s[16];
  auto load_group = [&](long long r, int g, float2* dst) {
    const float2* row = X + (size_t)r * N;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const float a = amp[g + R * (t + 256 * j)];
      const float2 x = row[g * 4096 + t + 256 * j];
      dst[j] = make_float2(x.x * a, x.y * a);
    }
  };
  if (r0 < r1) load_group(r0, h, s);
  for (long long r = r0; r < r1; ++r) {
    float2* row = X + (size_t)r * N;
#pragma unroll
    for (int i = 0; i < G; ++i) {
      const int g = h + H * i;
      float2* A = L + g * kFftLds;
      float2 v[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) v[j] = s[j];
      if (i + 1 < G) load_group(r, g + H, s);
      else if (r + 1 < r1) load_group(r + 1, h, s);
      fft_pass1_compute<true>(v, t, tw);
      __syncthreads();   // the previous group's or row's last LDS reads are done
      fft_pass1_store(v, t, A);
      __syncthreads();
      fft_pass2<true>(t, tw, A);
      __syncthreads();
      fft_pass3<true>(v, t, A);
      // this thread holds y_g[t + 256 j] of its group's 4096-point inverse
      if constexpr (R == 1) {
#pragma unroll
        for (int j = 0; j < 16; ++j) row[t + 256 * j] = v[j];
      } else {
        __syncthreads();   // every pass-3 read of this group is done
#pragma unroll
        for (int j = 0; j < 16; ++j) A[fft_lds(j, t >> 4, t & 15)] = v[j];
      }
    }
    if constexpr (R > 1) {
      __syncthreads();
      // the radix-R pass: x[n2 + 4096 n1] for this thread's n2 = T + NT m
#pragma unroll 2
      for (int m = 0; m < M; ++m) {
        const int n2 = T + NT * m;
        float2 u[R];
#pragma unroll
        for (int k1 = 0; k1 < R; ++k1) {
          const float2 y = L[k1 * kFftLds + fft_lds(n2 >> 8, (n2 >> 4) & 15, n2 & 15)];
          u[k1] = k1 == 0 ? y : fft_cmul(y, fft_tw<true>(tw, kFftTw + (k1 - 1) * 4096 + n2));
        }
        whiten_dftR<R, true>(u);
#pragma unroll
        for (int n1 = 0; n1 < R; ++n1) row[n2 + 4096 * n1] = u[n1];
      }
    }
  }
}

template <int R>
static int launch_whiten_hand(float2* X, long long rows, double gamma, unsigned char* work, hipStream_t st) {
  constexpr int N = 4096 * R;
  const int lds = R * kFftLds * (int)sizeof(float2);
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 3;
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(whiten_forward_kernel<R>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess ||
      hipFuncSetAttribute(reinterpret_cast<const void*>(whiten_inverse_kernel<R>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess)
    return 3;
  // row blocks (workgroups): the resident count, at most one row each, and
  // their partial sums within the buffer
  const long long nb = std::min<long long>(rows, std::min<long long>((long long)(kWhitenPartWords / N),
                                                                      (long long)cus * (4 / R)));
  double* part = reinterpret_cast<double*>(work);
  double* phat = part + kWhitenPartWords;
  float* amp = reinterpret_cast<float*>(phat + 16384);
  float2* tw = reinterpret_cast<float2*>(amp + 16384);
  hipLaunchKernelGGL(whiten_tables_kernel, dim3(16), dim3(kThreads), 0, st, tw, R);
  hipLaunchKernelGGL(whiten_forward_kernel<R>, dim3((unsigned)nb), dim3(whiten_threads<R>()), lds, st, X, rows,
                     (const float2*)tw, part);
  hipLaunchKernelGGL(whiten_estimate_kernel, dim3((N + kThreads - 1) / kThreads), dim3(kThreads), 0, st,
                     (const double*)part, (int)nb, rows, N, phat);
  hipLaunchKernelGGL(whiten_gain_kernel, dim3(1), dim3(kThreads), 0, st, N, gamma, (const double*)phat, amp);
  hipLaunchKernelGGL(whiten_inverse_kernel<R>, dim3((unsigned)nb), dim3(whiten_threads<R>()), lds, st, X, rows,
                     (const float2*)tw, (const float*)amp);
  return hipGetLastError() == hipSuccess ? 0 : 3;
}

// work: the larger of the two paths' needs. rocFFT path: kWhitenBlocks * Ns +
// Ns doubles, then Ns floats. Hand-written path: kWhitenPartWords + 16384
// doubles, 16384 floats, kWhitenTw float2.
size_t whiten_work_bytes(int Ns) {
  const size_t lib = sizeof(double) * ((size_t)kWhitenBlocks * Ns + Ns) + sizeof(float) * (size_t)Ns;
  const size_t hand = whiten_radix(Ns) ? sizeof(double) * (kWhitenPartWords + 16384) + sizeof(float) * 16384 +
                                           sizeof(float2) * kWhitenTw
                                       : 0;
  return std::max(lib, hand);
}

bool whiten_hand_written(int Ns) { return whiten_radix(Ns) != 0; }

int launch_whiten(void* fft_plan, void* echo, long long rows, int Ns, double gamma, void* work, hipStream_t st) {
  switch (whiten_radix(Ns)) {
    case 1: return launch_whiten_hand<1>(reinterpret_cast<float2*>(echo), rows, gamma, (unsigned char*)work, st);
    case 2: return launch_whiten_hand<2>(reinterpret_cast<float2*>(echo), rows, gamma, (unsigned char*)work, st);
    case 4: return launch_whiten_hand<4>(reinterpret_cast<float2*>(echo), rows, gamma, (unsigned char*)work, st);
    default: break;
  }
  hipfftHandle h = reinterpret_cast<hipfftHandle>(fft_plan);
  hipfftComplex* X = reinterpret_cast<hipfftComplex*>(echo);
  double* part = reinterpret_cast<double*>(work);
  double* phat = part + (size_t)kWhitenBlocks * Ns;
  float* amp = reinterpret_cast<float*>(phat + Ns);
  if (hipfftSetStream(h, st) != HIPFFT_SUCCESS) return 1;
  if (hipfftExecC2C(h, X, X, HIPFFT_FORWARD) != HIPFFT_SUCCESS) return 2;
  hipLaunchKernelGGL(whiten_power_kernel, dim3((Ns + kThreads - 1) / kThreads, kWhitenBlocks), dim3(kThreads), 0, st,
                     (const float2*)echo, rows, Ns, part);
  hipLaunchKernelGGL(whiten_estimate_kernel, dim3((Ns + kThreads - 1) / kThreads), dim3(kThreads), 0, st,
                     (const double*)part, kWhitenBlocks, rows, Ns, phat);
  hipLaunchKernelGGL(whiten_gain_kernel, dim3(1), dim3(kThreads), 0, st, Ns, gamma, (const double*)phat, amp);
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

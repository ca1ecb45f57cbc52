// Range compression and basebanding of an echo cube: the matched filter with
// the transmitted waveform q of Eq. 1 (Sec. II-A), which turns the received
// analytic signal into the compressed complex baseband echo the
// backprojection sum reads.
//
// Per (ping, element) row x[k] at t_k = t0 + k / f_s:
//     b[k] = x[k] exp(-j 2 pi f_c t_k)                  (when mixing)
//     y[n] = sum_{m<M} b[n + m] conj(q[m]) / sum_m |q[m]|^2,   b = 0 past N_s.
// Two fast-correlation forms, both with H = conj(Q) / (L E_q), Q the
// replica's L-point transform, E_q its energy:
//  * fused (M <= kRcFusedTaps): overlap-save with L = 4096. One workgroup per
//    row walks its segments in order; segment s reads b[sU, sU + 4096)
//    (U = 4097 - M useful outputs), transforms it in LDS, multiplies by H,
//    transforms back and writes y[sU, sU + U) over the input. Later segments
//    only read beyond what earlier ones wrote, so the row is done in place
//    with one HBM read (plus the (M - 1) / U overlap) and one write.
//  * batched (longer replicas): rows zero-padded to L >= N_s + M - 1 (so the
//    circular correlation does not wrap), transformed in batches of B rows
//    (rocFFT through hipFFT), multiplied by H, transformed back; the first
//    N_s samples are written over the input.
// The mix table and H are made once per call: the carrier phase in FP64
// (cycles reduced to [0, 1)), the replica energy summed in FP64 in a fixed
// order. A replica of zero energy gives an all-zero output.
#include <hipfft/hipfft.h>

#include "tdbp_dev.h"
#include "tdbp_fft.h"

namespace sasbp {

constexpr int kRcFusedTaps = 2048;   // longest replica of the fused form (U >= 2049 of 4096)

int rc_fused_taps() { return kRcFusedTaps; }

__global__ __launch_bounds__(kThreads) void rc_mix_kernel(float2* mix, int Ns, double fc, double t0, double fs,
                                                          int apply) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= Ns) return;
  if (!apply) {
    mix[k] = make_float2(1.0f, 0.0f);
    return;
  }
  const double cyc = fc * (t0 + (double)k / fs);
  const double fr = cyc - floor(cyc);
  double s, c;
  sincospi(-2.0 * fr, &s, &c);
  mix[k] = make_float2((float)c, (float)s);
}

// H[0..L) = replica zero-padded to L; energy = sum |q|^2 (FP64, fixed order).
__global__ __launch_bounds__(kThreads) void rc_replica_kernel(const float2* q, int M, int L, float2* H,
                                                              double* energy) {
  __shared__ double red[kThreads];
  double s = 0.0;
  for (int m = threadIdx.x; m < L; m += kThreads) {
    const float2 v = m < M ? q[m] : make_float2(0.0f, 0.0f);
    H[m] = v;
    s += (double)v.x * v.x + (double)v.y * v.y;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *energy = red[0];
}

// H <- conj(H) / (L E_q): the inverse transform's 1/L folded in.
__global__ __launch_bounds__(kThreads) void rc_filter_kernel(float2* H, int L, const double* energy) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= L) return;
  const double e = *energy;
  const float g = e > 0.0 ? (float)(1.0 / ((double)L * e)) : 0.0f;
  const float2 v = H[f];
  H[f] = make_float2(v.x * g, -v.y * g);
}

// buf[r][k] = x[row0 + r][k] mix[k] for k < N_s, 0 up to L and for rows past the cube.
__global__ __launch_bounds__(kThreads) void rc_load_kernel(const float2* x, long long row0, long long rows, int Ns,
                                                           int L, const float2* mix, float2* buf) {
  const long long row = row0 + blockIdx.y;
  float2* dst = buf + (size_t)blockIdx.y * L;
  const float2* src = x + (size_t)row * Ns;
  const bool live = row < rows;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < L; k += gridDim.x * blockDim.x) {
    float2 v = make_float2(0.0f, 0.0f);
    if (live && k < Ns) {
      const float2 a = src[k], w = mix[k];
      v = make_float2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
    }
    dst[k] = v;
  }
}

__global__ __launch_bounds__(kThreads) void rc_multiply_kernel(float2* buf, int L, const float2* H) {
  float2* row = buf + (size_t)blockIdx.y * L;
  for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < L; f += gridDim.x * blockDim.x) {
    const float2 a = row[f], h = H[f];
    row[f] = make_float2(a.x * h.x - a.y * h.y, a.x * h.y + a.y * h.x);
  }
}

__global__ __launch_bounds__(kThreads) void rc_store_kernel(const float2* buf, long long row0, long long rows, int Ns,
                                                            int L, float2* x) {
  const long long row = row0 + blockIdx.y;
  if (row >= rows) return;
  const float2* src = buf + (size_t)blockIdx.y * L;
  float2* dst = x + (size_t)row * Ns;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < Ns; k += gridDim.x * blockDim.x) dst[k] = src[k];
}

// The transform's twiddle table (from FP64), the replica energy and
// H = conj(Q) / (4096 E_q) for the fused form, in natural bin order. One
// workgroup.
__global__ __launch_bounds__(kFftThreads) void rc_spectrum_kernel(const float2* q, int M, float2* H, float2* tw,
                                                                  double* energy) {
  __shared__ float2 A[kFftLds];
  __shared__ float2 T[kFftTw];
  __shared__ double red[kFftThreads];
  const int t = threadIdx.x;
  for (int i = t; i < kFftTw; i += kFftThreads) {
    double sn, cs;
    sincospi(-2.0 * (double)fft_tw_exponent(i) / (double)kFftN, &sn, &cs);
    T[i] = make_float2((float)cs, (float)sn);
    tw[i] = T[i];
  }
  double e = 0.0;
  for (int m = t; m < M; m += kFftThreads) e += (double)q[m].x * q[m].x + (double)q[m].y * q[m].y;
  red[t] = e;
  float2 v[16];
#pragma unroll
  for (int n1 = 0; n1 < 16; ++n1) {
    const int m = n1 * kFftThreads + t;
    v[n1] = m < M ? q[m] : make_float2(0.0f, 0.0f);
  }
  __syncthreads();
  for (int h = kFftThreads / 2; h > 0; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  const double eq = red[0];
  fft_pass1_compute<false>(v, t, T);
  fft_pass1_store(v, t, A);
  __syncthreads();
  fft_pass2<false>(t, T, A);
  __syncthreads();
  fft_pass3<false>(v, t, A);
  const float g = eq > 0.0 ? (float)(1.0 / ((double)kFftN * eq)) : 0.0f;
#pragma unroll
  for (int j = 0; j < 16; ++j) H[t + kFftThreads * j] = make_float2(v[j].x * g, -v[j].y * g);
  if (t == 0) *energy = eq;
}

// Fused overlap-save correlation, in place; one workgroup per row (grid-stride).
__global__ __launch_bounds__(kFftThreads) void rc_fused_kernel(float2* x, long long rows, int Ns, int U, int nseg,
                                                               const float2* mix, const float2* H, const float2* tw) {
  __shared__ float2 A[kFftLds];
  __shared__ float2 T[kFftTw];
  const int t = threadIdx.x;
  for (int i = t; i < kFftTw; i += kFftThreads) T[i] = tw[i];
  __syncthreads();
  // the next segment's samples and mix factors, loaded while the current one
  // is transformed (a segment reads [s U, s U + 4096) and writes [s U, s U +
  // U): no later segment reads what an earlier one wrote)
  float2 nx[16], nm[16];
  auto load_seg = [&](long long row, int s) {
    const float2* xr = x + (size_t)row * Ns;
    const int i0 = s * U;
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) {
      const int i = i0 + n1 * kFftThreads + t;
      nx[n1] = i < Ns ? xr[i] : make_float2(0.0f, 0.0f);
      nm[n1] = i < Ns ? mix[i] : make_float2(0.0f, 0.0f);
    }
  };
  if (blockIdx.x < rows) load_seg(blockIdx.x, 0);
  for (long long row = blockIdx.x; row < rows; row += gridDim.x) {
    float2* xr = x + (size_t)row * Ns;
    for (int s = 0; s < nseg; ++s) {
      const int i0 = s * U;
      float2 v[16];
#pragma unroll
      for (int n1 = 0; n1 < 16; ++n1) v[n1] = fft_cmul(nx[n1], nm[n1]);
      if (s + 1 < nseg) load_seg(row, s + 1);
      else if (row + gridDim.x < rows) load_seg(row + gridDim.x, 0);
      fft_pass1_compute<false>(v, t, T);
      __syncthreads();   // the previous segment's last LDS reads are done
      fft_pass1_store(v, t, A);
      __syncthreads();
      fft_pass2<false>(t, T, A);
      __syncthreads();
      fft_pass3<false>(v, t, A);
#pragma unroll
      for (int j = 0; j < 16; ++j) v[j] = fft_cmul(v[j], H[t + kFftThreads * j]);
      fft_pass1_compute<true>(v, t, T);
      __syncthreads();
      fft_pass1_store(v, t, A);
      __syncthreads();
      fft_pass2<true>(t, T, A);
      __syncthreads();
      fft_pass3<true>(v, t, A);
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int n = t + kFftThreads * j;
        if (n < U && i0 + n < Ns) xr[i0 + n] = v[j];
      }
    }
  }
}

// Smallest L >= n whose only prime factors are 2, 3 and 5 (sizes rocFFT
// transforms without a Bluestein stage).
int rc_transform_length(long long n) {
  long long best = 1;
  while (best < n) best <<= 1;
  for (long long p5 = 1; p5 < best; p5 *= 5)
    for (long long p35 = p5; p35 < best; p35 *= 3) {
      long long v = p35;
      while (v < n) v <<= 1;
      if (v < best) best = v;
    }
  return best > 0x7fffffffll ? -1 : (int)best;
}

int rc_make_plans(int L, int B, void** batch, void** single) {
  hipfftHandle hb, hs;
  if (hipfftPlan1d(&hb, L, HIPFFT_C2C, B) != HIPFFT_SUCCESS) return 1;
  if (hipfftPlan1d(&hs, L, HIPFFT_C2C, 1) != HIPFFT_SUCCESS) {
    (void)hipfftDestroy(hb);
    return 1;
  }
  *batch = reinterpret_cast<void*>(hb);
  *single = reinterpret_cast<void*>(hs);
  return 0;
}

static dim3 row_grid(int n, int rows) {
  int bx = (n + kThreads - 1) / kThreads;
  if (bx > 16) bx = 16;   // a few row segments per workgroup keep the grid modest
  return dim3((unsigned)bx, (unsigned)rows);
}

int launch_range_compress_fused(void* echo, long long rows, int Ns, const void* replica, int M, double fc, double t0,
                                double fs, int apply_mix, void* filt, void* tw, void* mixtab, void* energy,
                                hipStream_t st) {
  const int U = kFftN + 1 - M;
  const int nseg = (Ns + U - 1) / U;
  hipLaunchKernelGGL(rc_mix_kernel, dim3((Ns + kThreads - 1) / kThreads), dim3(kThreads), 0, st,
                     reinterpret_cast<float2*>(mixtab), Ns, fc, t0, fs, apply_mix);
  hipLaunchKernelGGL(rc_spectrum_kernel, dim3(1), dim3(kFftThreads), 0, st, (const float2*)replica, M,
                     reinterpret_cast<float2*>(filt), reinterpret_cast<float2*>(tw),
                     reinterpret_cast<double*>(energy));
  const long long grid = rows < (1ll << 20) ? rows : (1ll << 20);
  hipLaunchKernelGGL(rc_fused_kernel, dim3((unsigned)grid), dim3(kFftThreads), 0, st,
                     reinterpret_cast<float2*>(echo), rows, Ns, U, nseg, (const float2*)mixtab, (const float2*)filt,
                     (const float2*)tw);
  return hipGetLastError() == hipSuccess ? 0 : 3;
}

// work: B L float2 rows, then L float2 filter, N_s float2 mix table, one double.
int launch_range_compress(void* batch_plan, void* single_plan, void* echo, long long rows, int Ns, int L, int B,
                          const void* replica, int M, double fc, double t0, double fs, int apply_mix, void* buf,
                          void* filt, void* mixtab, void* energy, hipStream_t st) {
  hipfftHandle hb = reinterpret_cast<hipfftHandle>(batch_plan);
  hipfftHandle hs = reinterpret_cast<hipfftHandle>(single_plan);
  float2* X = reinterpret_cast<float2*>(echo);
  float2* W = reinterpret_cast<float2*>(buf);
  float2* H = reinterpret_cast<float2*>(filt);
  float2* mix = reinterpret_cast<float2*>(mixtab);
  double* eq = reinterpret_cast<double*>(energy);
  if (hipfftSetStream(hb, st) != HIPFFT_SUCCESS || hipfftSetStream(hs, st) != HIPFFT_SUCCESS) return 1;
  hipLaunchKernelGGL(rc_mix_kernel, dim3((Ns + kThreads - 1) / kThreads), dim3(kThreads), 0, st, mix, Ns, fc, t0, fs,
                     apply_mix);
  hipLaunchKernelGGL(rc_replica_kernel, dim3(1), dim3(kThreads), 0, st, (const float2*)replica, M, L, H, eq);
  if (hipGetLastError() != hipSuccess) return 3;
  hipfftComplex* Hc = reinterpret_cast<hipfftComplex*>(H);
  if (hipfftExecC2C(hs, Hc, Hc, HIPFFT_FORWARD) != HIPFFT_SUCCESS) return 2;
  hipLaunchKernelGGL(rc_filter_kernel, dim3((L + kThreads - 1) / kThreads), dim3(kThreads), 0, st, H, L,
                     (const double*)eq);
  hipfftComplex* Wc = reinterpret_cast<hipfftComplex*>(W);
  for (long long row0 = 0; row0 < rows; row0 += B) {
    hipLaunchKernelGGL(rc_load_kernel, row_grid(L, B), dim3(kThreads), 0, st, (const float2*)X, row0, rows, Ns, L,
                       (const float2*)mix, W);
    if (hipGetLastError() != hipSuccess) return 3;
    if (hipfftExecC2C(hb, Wc, Wc, HIPFFT_FORWARD) != HIPFFT_SUCCESS) return 2;
    hipLaunchKernelGGL(rc_multiply_kernel, row_grid(L, B), dim3(kThreads), 0, st, W, L, (const float2*)H);
    if (hipGetLastError() != hipSuccess) return 3;
    if (hipfftExecC2C(hb, Wc, Wc, HIPFFT_BACKWARD) != HIPFFT_SUCCESS) return 2;
    hipLaunchKernelGGL(rc_store_kernel, row_grid(Ns, B), dim3(kThreads), 0, st, (const float2*)W, row0, rows, Ns, L,
                       X);
    if (hipGetLastError() != hipSuccess) return 3;
  }
  return 0;
}

}  // namespace sasbp

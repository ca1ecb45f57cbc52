// Time-delay estimation between consecutive pings for the displaced-phase-
// centre (DPC) motion estimate (Sec. II-D: the measured delay of Eq. 4 from
// overlapped coherent looks of the seafloor; coarse delay from quadratic
// interpolation of the correlation magnitude, phase at the interpolated point).
//
// One workgroup per (window k, ping pair i). For each of the J element pairs
// (e1 of ping i, e2 of ping i + 1) the window a = echo[i][e1][n0, n0 + W) and
// the lag-extended window b = echo[i + 1][e2][n0 - L, n0 + W + L) (zero outside
// the record) go to LDS; wave w accumulates the lags w, w + 4, ...:
//     r(l) += sum_n a[n] conj(b[n + l]),  eb(l) += sum_n |b[n + l]|^2
// (lanes split n, then a wave reduction), in FP32. The peak search, the
// quadratic step mu = (m_- - m_+) / (2 (m_- - 2 m_0 + m_+)) (0 on a flat top),
// the complex correlation at l* + mu and rho = |r(l*)| / sqrt(ea eb(l*)) are
// then formed in FP64 by one thread. The peak is the first maximum of |r| over
// |l| < L (both neighbours exist).
#include "tdbp_dev.h"

namespace sasbp {

constexpr int kTdeThreads = 256;
constexpr int kTdeMaxLag = 64;
constexpr int kTdeMaxLags = 2 * kTdeMaxLag + 1;

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(kTdeThreads) void dpc_tde_kernel(const float2* __restrict__ echo, int E, int Ns,
                                                              const int2* __restrict__ pairs, int J, int W, int hop,
                                                              int L, double fs, float4* __restrict__ out, int K) {
  extern __shared__ float2 tde_lds[];
  __shared__ float2 r_acc[kTdeMaxLags];
  __shared__ float eb_acc[kTdeMaxLags];
  __shared__ float ea_part[kTdeThreads / 64];
  const int k = blockIdx.x, i = blockIdx.y;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int NL = 2 * L + 1;
  const int n0 = k * hop;
  float2* sa = tde_lds;
  float2* sb = tde_lds + W;
  for (int li = t; li < NL; li += kTdeThreads) {
    r_acc[li] = make_float2(0.0f, 0.0f);
    eb_acc[li] = 0.0f;
  }
  float ea = 0.0f;
  for (int j = 0; j < J; ++j) {
    __syncthreads();   // the previous pair's LDS reads are done (and the accumulators cleared)
    const int2 pr = pairs[j];
    const float2* ra = echo + ((size_t)i * E + pr.x) * (size_t)Ns;
    const float2* rb = echo + ((size_t)(i + 1) * E + pr.y) * (size_t)Ns;
    for (int n = t; n < W; n += kTdeThreads) {
      const float2 v = ra[n0 + n];
      sa[n] = v;
      ea = fmaf(v.x, v.x, fmaf(v.y, v.y, ea));
    }
    for (int m = t; m < W + 2 * L; m += kTdeThreads) {
      const int idx = n0 - L + m;
      sb[m] = (idx >= 0 && idx < Ns) ? rb[idx] : make_float2(0.0f, 0.0f);
    }
    __syncthreads();
    for (int li = wave; li < NL; li += kTdeThreads / 64) {
      float re = 0.0f, im = 0.0f, e = 0.0f;
      for (int n = lane; n < W; n += 64) {
        const float2 a = sa[n], b = sb[n + li];
        re = fmaf(a.x, b.x, fmaf(a.y, b.y, re));
        im = fmaf(a.y, b.x, fmaf(-a.x, b.y, im));
        e = fmaf(b.x, b.x, fmaf(b.y, b.y, e));
      }
      re = wave_sum(re);
      im = wave_sum(im);
      e = wave_sum(e);
      if (lane == 0) {
        r_acc[li].x += re;
        r_acc[li].y += im;
        eb_acc[li] += e;
      }
    }
  }
  ea = wave_sum(ea);
  if (lane == 0) ea_part[wave] = ea;
  __syncthreads();
  if (t == 0) {
    double ea_tot = 0.0;
    for (int w = 0; w < kTdeThreads / 64; ++w) ea_tot += (double)ea_part[w];
    int ic = 1;
    double best = -1.0;
    for (int li = 1; li < NL - 1; ++li) {
      const double m = sqrt((double)r_acc[li].x * r_acc[li].x + (double)r_acc[li].y * r_acc[li].y);
      if (m > best) {
        best = m;
        ic = li;
      }
    }
    const double rmx = r_acc[ic - 1].x, rmy = r_acc[ic - 1].y;
    const double r0x = r_acc[ic].x, r0y = r_acc[ic].y;
    const double rpx = r_acc[ic + 1].x, rpy = r_acc[ic + 1].y;
    const double m_ = sqrt(rmx * rmx + rmy * rmy), mp = sqrt(rpx * rpx + rpy * rpy);
    const double den = m_ - 2.0 * best + mp;
    const double mu = den == 0.0 ? 0.0 : (m_ - mp) / (2.0 * den);
    const double cx = r0x + mu * (rpx - rmx) * 0.5 + mu * mu * (rpx - 2.0 * r0x + rmx) * 0.5;
    const double cy = r0y + mu * (rpy - rmy) * 0.5 + mu * mu * (rpy - 2.0 * r0y + rmy) * 0.5;
    const double d = sqrt(ea_tot * (double)eb_acc[ic]);
    const double rho = d > 0.0 ? best / d : 0.0;
    out[(size_t)i * K + k] = make_float4((float)(((double)(ic - L) + mu) / fs), (float)atan2(cy, cx), (float)rho,
                                         (float)(ic - L));
  }
}

int tde_max_lag() { return kTdeMaxLag; }

size_t tde_lds_bytes(int W, int L) { return sizeof(float2) * (size_t)(2 * W + 2 * L); }

hipError_t launch_dpc_tde(const void* echo, int P, int E, int Ns, const int* pairs, int J, int W, int hop, int L,
                          double fs, float* out, hipStream_t st) {
  const int K = (Ns - W) / hop + 1;
  hipLaunchKernelGGL(dpc_tde_kernel, dim3((unsigned)K, (unsigned)(P - 1)), dim3(kTdeThreads), tde_lds_bytes(W, L), st,
                     reinterpret_cast<const float2*>(echo), E, Ns, reinterpret_cast<const int2*>(pairs), J, W, hop,
                     L, fs, reinterpret_cast<float4*>(out), K);
  return hipGetLastError();
}

}  // namespace sasbp

// Time-delay estimation between consecutive pings for the displaced-phase-
// centre (DPC) motion estimate (Sec. II-D: the measured delay of Eq. 4 from
// overlapped coherent looks of the seafloor; coarse delay from quadratic
// interpolation of the correlation magnitude, phase at the interpolated point).
//
// One workgroup per (window k, ping pair i). The element pairs go through LDS
// in groups of G: for each pair j of a group, the window a = echo[i][e1][n0,
// n0 + W) and the lag-extended window b = echo[i + 1][e2][n0 - L, n0 + W + L)
// (zero outside the record). One thread owns a (pair, block of kTdeBlock
// lags, third of the samples) and forms its sums in registers, sliding a
// window of b values along n (two LDS reads per sample for kTdeBlock lags):
//     r(l) = sum_n a[n] conj(b[n + l]),  eb(l) = sum_n |b[n + l]|^2   (FP32)
// then the group's partial sums are added per lag over pairs and sample
// thirds, in a fixed order.
// The peak search, the quadratic step mu = (m_- - m_+) / (2 (m_- - 2 m_0 +
// m_+)) (0 on a flat top), the complex correlation at l* + mu and rho =
// |r(l*)| / sqrt(ea eb(l*)) are then formed in FP64 by one thread. The peak
// is the first maximum of |r| over |l| < L (both neighbours exist).
#include "tdbp_dev.h"

namespace sasbp {

constexpr int kTdeThreads = 256;
constexpr int kTdeMaxLag = 64;
constexpr int kTdeMaxLags = 2 * kTdeMaxLag + 1;
constexpr int kTdeBlock = 4;             // lags per thread
constexpr int kTdeLdsTarget = 24576;     // bytes of looks per group (several workgroups per CU)
constexpr int kTdeSplit = 3;             // sample segments per (pair, lag block), summed in LDS

// Pairs per LDS group for windows of W samples and lags to +-L.
__host__ __device__ inline int tde_group(int W, int L, int J) {
  const int per = (2 * W + 2 * L + kTdeBlock) * 8 + kTdeSplit * (2 * L + 1) * 12;
  int g = kTdeLdsTarget / per;
  g = g < 1 ? 1 : g;
  return g < J ? g : J;
}

__global__ __launch_bounds__(kTdeThreads) void dpc_tde_kernel(const float2* __restrict__ echo, int E, int Ns,
                                                              const int2* __restrict__ pairs, int J, int W, int hop,
                                                              int L, double fs, float4* __restrict__ out, int K) {
  extern __shared__ __align__(16) unsigned char tde_lds[];
  __shared__ float2 r_acc[kTdeMaxLags];
  __shared__ float eb_acc[kTdeMaxLags];
  __shared__ float ea_acc;
  const int k = blockIdx.x, i = blockIdx.y;
  const int t = threadIdx.x;
  const int NL = 2 * L + 1;
  const int NB = (NL + kTdeBlock - 1) / kTdeBlock;
  const int WB = W + 2 * L + kTdeBlock;   // b window with zero tail for the last lag block
  const int n0 = k * hop;
  const int G = tde_group(W, L, J);
  float2* sa = reinterpret_cast<float2*>(tde_lds);            // [G][W]
  float2* sb = sa + (size_t)G * W;                            // [G][WB]
  float2* pr_r = sb + (size_t)G * WB;                         // [kTdeSplit][G][NL]
  float* pr_e = reinterpret_cast<float*>(pr_r + (size_t)kTdeSplit * G * NL);   // [kTdeSplit][G][NL]
  const int WS = (W + kTdeSplit - 1) / kTdeSplit;             // samples per segment
  for (int li = t; li < NL; li += kTdeThreads) {
    r_acc[li] = make_float2(0.0f, 0.0f);
    eb_acc[li] = 0.0f;
  }
  if (t == 0) ea_acc = 0.0f;
  for (int g0 = 0; g0 < J; g0 += G) {
    const int gJ = min(G, J - g0);
    __syncthreads();   // the previous group's LDS reads are done (and the accumulators cleared)
    for (int j = 0; j < gJ; ++j) {
      const int2 pr = pairs[g0 + j];
      const float2* ra = echo + ((size_t)i * E + pr.x) * (size_t)Ns;
      const float2* rb = echo + ((size_t)(i + 1) * E + pr.y) * (size_t)Ns;
      for (int n = t; n < W; n += kTdeThreads) sa[j * W + n] = ra[n0 + n];
      for (int m = t; m < WB; m += kTdeThreads) {
        const int idx = n0 - L + m;
        sb[j * WB + m] = (m < W + 2 * L && idx >= 0 && idx < Ns) ? rb[idx] : make_float2(0.0f, 0.0f);
      }
    }
    __syncthreads();
    if (t < 64) {   // window energy of this group's first looks, one wave, pair order
      float e = 0.0f;
      for (int j = 0; j < gJ; ++j)
        for (int n = t; n < W; n += 64) {
          const float2 v = sa[j * W + n];
          e = fmaf(v.x, v.x, fmaf(v.y, v.y, e));
        }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o, 64);
      if (t == 0) ea_acc += e;
    }
    for (int it = t; it < kTdeSplit * gJ * NB; it += kTdeThreads) {
      const int seg = it / (gJ * NB), jt = it - seg * gJ * NB;
      const int j = jt / NB, l0 = (jt - j * NB) * kTdeBlock;
      const int nlo = seg * WS, nhi = min(W, nlo + WS);
      const float2* a = sa + j * W;
      const float2* b = sb + j * WB + l0;
      float re[kTdeBlock], im[kTdeBlock], en[kTdeBlock];
      float2 bw[kTdeBlock];
#pragma unroll
      for (int r = 0; r < kTdeBlock; ++r) {
        re[r] = im[r] = en[r] = 0.0f;
        bw[r] = b[nlo + r];
      }
      for (int n = nlo; n < nhi; ++n) {
        const float2 av = a[n];
#pragma unroll
        for (int r = 0; r < kTdeBlock; ++r) {   // a[n] conj(b[n + l])
          re[r] = fmaf(av.x, bw[r].x, fmaf(av.y, bw[r].y, re[r]));
          im[r] = fmaf(av.y, bw[r].x, fmaf(-av.x, bw[r].y, im[r]));
          en[r] = fmaf(bw[r].x, bw[r].x, fmaf(bw[r].y, bw[r].y, en[r]));
        }
#pragma unroll
        for (int r = 0; r < kTdeBlock - 1; ++r) bw[r] = bw[r + 1];
        bw[kTdeBlock - 1] = b[n + kTdeBlock];
      }
#pragma unroll
      for (int r = 0; r < kTdeBlock; ++r)
        if (l0 + r < NL) {
          pr_r[(seg * G + j) * NL + l0 + r] = make_float2(re[r], im[r]);
          pr_e[(seg * G + j) * NL + l0 + r] = en[r];
        }
    }
    __syncthreads();
    for (int li = t; li < NL; li += kTdeThreads) {
      float2 racc = r_acc[li];
      float eacc = eb_acc[li];
      for (int j = 0; j < gJ; ++j)
        for (int sg = 0; sg < kTdeSplit; ++sg) {
          racc.x += pr_r[(sg * G + j) * NL + li].x;
          racc.y += pr_r[(sg * G + j) * NL + li].y;
          eacc += pr_e[(sg * G + j) * NL + li];
        }
      r_acc[li] = racc;
      eb_acc[li] = eacc;
    }
  }
  __syncthreads();
  if (t == 0) {
    const double ea_tot = (double)ea_acc;
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

size_t tde_lds_bytes(int W, int L, int J) {
  const int G = tde_group(W, L, J);
  return (size_t)G * ((size_t)(2 * W + 2 * L + kTdeBlock) * 8 + (size_t)kTdeSplit * (2 * L + 1) * 12);
}

hipError_t launch_dpc_tde(const void* echo, int P, int E, int Ns, const int* pairs, int J, int W, int hop, int L,
                          double fs, float* out, hipStream_t st) {
  const int K = (Ns - W) / hop + 1;
  hipLaunchKernelGGL(dpc_tde_kernel, dim3((unsigned)K, (unsigned)(P - 1)), dim3(kTdeThreads), tde_lds_bytes(W, L, J), st,
                     reinterpret_cast<const float2*>(echo), E, Ns, reinterpret_cast<const int2*>(pairs), J, W, hop,
                     L, fs, reinterpret_cast<float4*>(out), K);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Motion estimate from the measured delays (Eqs. 3-8, Sec. II-D): the Eq. 4
// residual of every (ping pair i, window k) and its derivatives, FP64 (the
// path differences are millimetres of paths tens of metres long). With the
// ping's platform position P_i = p_0 + sum_{n<i} v_n dt_n, TX = P + l_T and
// RX_e(t) = P + v t + l_e, and u(X) = (X - p_s) / |X - p_s|:
//   c J g = sum_j |TX_1 - p_s| + |p_s - RX_1j(t)| - |TX_2 - p_s| - |p_s - RX_2j(t)|  (+ c J delta)
//   dg/dP_i     = a = sum_j u(TX_1) + u(RX_1j) - u(TX_2) - u(RX_2j)      / (c J)
//   dg/dv_i     = b = sum_j t u(RX_1j) - dt_i (u(TX_2) + u(RX_2j))      / (c J)
//   dg/dv_{i+1} = d = -sum_j t u(RX_2j)                                 / (c J)
// (dg/dv_n = dt_n a for n < i). Output per row: g, a_y, a_z, b_y, b_z, d_y, d_z.
__global__ __launch_bounds__(kThreads) void dpc_residual_kernel(
    int P, int K, int J, const double* __restrict__ pos, const double* __restrict__ vel,
    const double* __restrict__ dt, double ltx, double lty, double ltz, const double* __restrict__ lever_rx,
    const int2* __restrict__ pairs, const double* __restrict__ t_ref, const double* __restrict__ ps,
    const double* __restrict__ delay, double c, double* __restrict__ rows) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= (long long)(P - 1) * K) return;
  const int i = (int)(r / K), k = (int)(r - (long long)i * K);
  const double t = t_ref[k];
  const double* s = ps + (size_t)r * 3;
  const double* P1 = pos + (size_t)i * 3;
  const double* P2 = pos + (size_t)(i + 1) * 3;
  const double* V1 = vel + (size_t)i * 3;
  const double* V2 = vel + (size_t)(i + 1) * 3;
  const double dti = dt[i];
  double tx1[3] = {P1[0] + ltx, P1[1] + lty, P1[2] + ltz};
  double tx2[3] = {P2[0] + ltx, P2[1] + lty, P2[2] + ltz};
  double u1[3], u2[3];
  const double d1 = sqrt((tx1[0] - s[0]) * (tx1[0] - s[0]) + (tx1[1] - s[1]) * (tx1[1] - s[1]) +
                         (tx1[2] - s[2]) * (tx1[2] - s[2]));
  const double d2 = sqrt((tx2[0] - s[0]) * (tx2[0] - s[0]) + (tx2[1] - s[1]) * (tx2[1] - s[1]) +
                         (tx2[2] - s[2]) * (tx2[2] - s[2]));
  for (int a = 0; a < 3; ++a) {
    u1[a] = (tx1[a] - s[a]) / d1;
    u2[a] = (tx2[a] - s[a]) / d2;
  }
  double path = 0.0, A[3] = {0.0, 0.0, 0.0}, B[3] = {0.0, 0.0, 0.0}, D[3] = {0.0, 0.0, 0.0};
  for (int j = 0; j < J; ++j) {
    const int2 pr = pairs[j];
    const double* l1 = lever_rx + (size_t)pr.x * 3;
    const double* l2 = lever_rx + (size_t)pr.y * 3;
    double x1[3], x2[3];
    for (int a = 0; a < 3; ++a) {
      x1[a] = P1[a] + V1[a] * t + l1[a] - s[a];
      x2[a] = P2[a] + V2[a] * t + l2[a] - s[a];
    }
    const double e1 = sqrt(x1[0] * x1[0] + x1[1] * x1[1] + x1[2] * x1[2]);
    const double e2 = sqrt(x2[0] * x2[0] + x2[1] * x2[1] + x2[2] * x2[2]);
    path += (d1 + e1) - (d2 + e2);
    for (int a = 0; a < 3; ++a) {
      const double w1 = x1[a] / e1, w2 = x2[a] / e2;
      A[a] += u1[a] + w1 - u2[a] - w2;
      B[a] += t * w1 - dti * (u2[a] + w2);
      D[a] -= t * w2;
    }
  }
  const double f = 1.0 / (c * (double)J);
  double* o = rows + (size_t)r * 7;
  o[0] = path * f + delay[r];
  o[1] = A[1] * f;
  o[2] = A[2] * f;
  o[3] = B[1] * f;
  o[4] = B[2] * f;
  o[5] = D[1] * f;
  o[6] = D[2] * f;
}

hipError_t launch_dpc_residual(int P, int K, int J, const double* pos, const double* vel, const double* dt,
                               const double* lever_tx, const double* lever_rx, const int* pairs, const double* t_ref,
                               const double* ps, const double* delay, double c, double* rows, hipStream_t st) {
  const long long n = (long long)(P - 1) * K;
  hipLaunchKernelGGL(dpc_residual_kernel, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, P,
                     K, J, pos, vel, dt, lever_tx[0], lever_tx[1], lever_tx[2], lever_rx,
                     reinterpret_cast<const int2*>(pairs), t_ref, ps, delay, c, rows);
  return hipGetLastError();
}

}  // namespace sasbp

namespace sasbp {

// Fine delay of every (ping pair, window) (Sec. II-D, the second step): the
// phase of the correlation at the coarse peak, phi = 2 pi f_c delta (mod 2 pi),
// unwrapped to the whole number of carrier cycles that brings it nearest the
// delay predicted by a first motion solution. rows are the Eq. 4 residual rows
// of that solution evaluated with a zero measured delay, so that rows[7 r] =
// c^-1 mean_j (path_1 - path_2) and the predicted delay is its negative:
//     m = round(f_c ref - phi / 2 pi),  delta = (phi + 2 pi m) / (2 pi f_c).
__global__ __launch_bounds__(kThreads) void dpc_fine_delay_kernel(long long n, const float4* __restrict__ tde,
                                                                 const double* __restrict__ rows, double fc,
                                                                 double* __restrict__ out) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const double two_pi = 6.283185307179586;
  const double phi = (double)tde[r].y;
  const double ref = -rows[(size_t)r * 7];
  const double m = rint(fc * ref - phi / two_pi);
  out[r] = (phi + two_pi * m) / (two_pi * fc);
}

hipError_t launch_dpc_fine_delay(long long n, const float* tde, const double* rows, double fc, double* out,
                                 hipStream_t st) {
  hipLaunchKernelGGL(dpc_fine_delay_kernel, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, n,
                     reinterpret_cast<const float4*>(tde), rows, fc, out);
  return hipGetLastError();
}

// p_i(0) = p_0 + sum_{n<i} v_n dt_n for every ping (one thread, in ping order).
__global__ void dpc_positions_kernel(int P, const double* __restrict__ vel, const double* __restrict__ dt, double p0x,
                                     double p0y, double p0z, double* __restrict__ pos) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double x = p0x, y = p0y, z = p0z;
  for (int i = 0; i < P; ++i) {
    pos[3 * i] = x;
    pos[3 * i + 1] = y;
    pos[3 * i + 2] = z;
    if (i + 1 < P) {
      x += vel[3 * i] * dt[i];
      y += vel[3 * i + 1] * dt[i];
      z += vel[3 * i + 2] * dt[i];
    }
  }
}

hipError_t launch_dpc_positions(int P, const double* vel, const double* dt, const double* p0, double* pos,
                                hipStream_t st) {
  hipLaunchKernelGGL(dpc_positions_kernel, dim3(1), dim3(64), 0, st, P, vel, dt, p0[0], p0[1], p0[2], pos);
  return hipGetLastError();
}

}  // namespace sasbp

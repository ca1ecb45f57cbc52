// Image formation: cull -> cost ordering -> persistent backprojection.
//
// Backprojection (Eq. 1 inverted per pixel, Sec. II-A) with pixel-stationary
// accumulation: a workgroup owns one tile of pixels at a time and keeps its
// complex sums in registers across every ping, so each pixel is written once
// (the paper's ping-outer loop re-reads and re-writes the image per ping).
// Pixels are independent (Sec. II-A), so tiles need no atomics and any
// processing order gives bitwise identical images.
//
// For each run of pings of its tile the workgroup forms, all threads at once,
// the FP64 reference geometry of every (ping, element) and, with a beam gate,
// the exact per-row gate intervals (Sec. II-C; transmitter and receiver
// tested separately as in the bistatic case, Sec. III-B), into its own
// region of the workspace. Then, per chunk of consecutive (ping, element)
// records of the run (part of a ping, one ping or several, sized so that
// three workgroups share a CU), it
//   1. copies the chunk's records and gate rows into LDS;
//   2. copies each (ping, element)'s echo window into LDS with coalesced loads,
//      zero-filling samples outside the record and converting FP16/BF16
//      storage to FP32;
//   3. updates K pixels per lane per (ping, element): FP32 delay offset,
//      linear (or windowed-sinc) interpolation from LDS, carrier phase via the
//      hardware sin/cos (which take revolutions), complex multiply-accumulate.
#include "tdbp_geom.h"

namespace sasbp {

__global__ void init_kernel(Workspace ws) {
  const int t = threadIdx.x;
  if (t == 0) ws.counters[0] = 0u;
  if (t < kXcds) ws.counters[kQueueCursor + t] = 0u;
  if (t < kBuckets) ws.bucket[t] = 0u;
}


// Conservative per-(tile, ping) test: can any pixel of the tile box lie inside
// the transmit cone and the cone of some element, and can its delay fall in
// the record? Keeps a superset of the exact set; the image kernel applies the
// exact per-row test, so the cull never changes a pixel. With the cull off
// (no_cull) every ping is kept.
__global__ __launch_bounds__(kThreads) void cull_kernel(Workspace ws, int TX, int TY, int TZ, int bucket_shift) {
  const int t = blockIdx.x;
  const int s = __builtin_amdgcn_readfirstlane(ws.tile_swath[t]);
  const SwathDev& sw = ws.swaths[s];
  const int lt = t - sw.tile0;
  const int ix = lt % sw.ntx, iy = (lt / sw.ntx) % sw.nty, iz = lt / (sw.ntx * sw.nty);
  const double xa = sw.o[0] + (double)(ix * TX) * sw.d[0], xb = xa + (double)(TX - 1) * sw.d[0];
  const double ya = sw.o[1] + (double)(iy * TY) * sw.d[1], yb = ya + (double)(TY - 1) * sw.d[1];
  const double za = sw.o[2] + (double)(iz * TZ) * sw.d[2], zb = za + (double)(TZ - 1) * sw.d[2];
  const double C[3] = {0.5 * (xa + xb), 0.5 * (ya + yb), 0.5 * (za + zb)};
  const double c = *sw.c;
  const bool c_ok = isfinite(c) && c >= sw.c_min;
  __shared__ int s_lo, s_hi;
  if (threadIdx.x == 0) { s_lo = 0x7fffffff; s_hi = -1; }
  __syncthreads();
  if (c_ok) {
    for (int p = threadIdx.x; p < sw.P; p += blockDim.x) {
      const double* T = sw.tx + (size_t)p * 3;
      // record test: the two-way delay of the tile lies within [dT0+dR0 - 2r, dT0+dR0 + 2r]
      const double u0 = C[0] - T[0], u1 = C[1] - T[1], u2 = C[2] - T[2];
      const double dT = sqrt(u0 * u0 + u1 * u1 + u2 * u2);
      // continuous motion moves a delay by at most the receiver's displacement:
      // |v| tau for a velocity, the table's largest one over the record (with
      // the line's departure from the table) for a table
      double vm = 0.0, dmax = 0.0;
      if (sw.motion == 1) {
        const double* V = sw.vel + (size_t)p * 3;
        vm = sqrt(V[0] * V[0] + V[1] * V[1] + V[2] * V[2]);
      } else if (sw.motion == 2) {
        const float4 st = sw.tstats[p];
        dmax = st.w == 0.0f ? (double)st.x * (1.0 + 1e-6) + 1e-5 : __builtin_nan("");
      }
      // the ping is kept when its transmitter's cone may hit the tile and one
      // element's cone and record both may (the elements are not tested
      // once the transmitter misses, nor after the first that passes)
      const bool tx_hit = !(sw.tan_g > 0.0 && !sw.no_cull) || cone_may_hit(sw.tan_g, xa, xb, ya, yb, za, zb, T);
      bool in_record = false;
      for (int e = 0; tx_hit && !in_record && e < sw.E; ++e) {
        const double* R = sw.rx + ((size_t)p * sw.E + e) * 3;
        const double v0 = C[0] - R[0], v1 = C[1] - R[1], v2 = C[2] - R[2];
        const double dR = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
        const double ulo = ((dT + dR - 2.0 * sw.half_diag) / c - sw.t0) * sw.fs;
        const double uhi = ((dT + dR + 2.0 * sw.half_diag) / c - sw.t0) * sw.fs;
        double reach = sw.interp == 1 ? (double)kSincHalf : 0.0;   // taps beyond the delay
        if (sw.motion == 1) reach += vm * (dT + dR + 2.0 * sw.half_diag) / c * sw.fs / c + 1.0;
        if (sw.motion == 2) reach += dmax * sw.fs / c + 1.0;
        // refracted legs are not straight: the record test is left to the kernel
        const bool rec_e = sw.refract || sw.no_cull ||
                           ((uhi >= -2.0 - reach) && (ulo <= (double)sw.Ns + 1.0 + reach));
        const bool gate_e = (sw.tan_g > 0.0 && !sw.no_cull) ? cone_may_hit(sw.tan_g, xa, xb, ya, yb, za, zb, R) : true;
        in_record = rec_e && gate_e;
      }
      // non-finite navigation makes every comparison false; keep such pings so
      // that the image kernel can flag them
      const bool bad = !(isfinite(dT)) || !isfinite(vm) || !isfinite(dmax);
      if ((tx_hit && in_record) || bad) {
        atomicMin(&s_lo, p);
        atomicMax(&s_hi, p);
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    PingRange pr;
    pr.lo = s_lo;
    pr.hi = s_hi;
    if (!c_ok) { pr.lo = 1; pr.hi = 0; atomicOr(&ws.counters[1], kStatusNav); }
    ws.prange[t] = pr;
    const long long npe = (pr.hi >= pr.lo) ? (long long)(pr.hi - pr.lo + 1) * sw.E : 0;
    int b = (int)(npe >> bucket_shift);
    b = b > kBuckets - 1 ? kBuckets - 1 : b;
    atomicAdd(&ws.bucket[b], 1u);
  }
}

// Position tables (motion 2): per ping, over the delays a record can hold
// (t in [0, t_end], t_end the end of the record plus two windows), the
// largest displacement |Delta(t)| (at a sample or at t_end, Delta being
// piecewise linear), the largest velocity change between neighbouring
// segments, the largest segment speed, and a flag for values that are not
// finite. One workgroup per ping; maxima of non-negative floats through
// their bit patterns.
__global__ __launch_bounds__(kThreads) void track_stats_kernel(Workspace ws, int s) {
  const SwathDev& sw = ws.swaths[s];
  const int p = blockIdx.x;
  const int N = sw.track_n;
  const double h = sw.track_h;
  const double t_end = sw.t0 + (double)(sw.Ns + 2 * sw.W + 4) / sw.fs;
  const double* a = sw.track + (size_t)p * N * 3;
  // samples up to the last one at or before t_end, and the segment past it
  const int jl = (int)fmin((double)(N - 1), fmax(1.0, floor(t_end / h) + 1.0));
  __shared__ unsigned s_max[4];
  if (threadIdx.x < 4) s_max[threadIdx.x] = 0u;
  __syncthreads();
  unsigned m0 = 0u, m1 = 0u, m2 = 0u, bad = 0u;
  for (int j = threadIdx.x; j <= jl; j += blockDim.x) {
    const double x = a[3 * j], y = a[3 * j + 1], z = a[3 * j + 2];
    bad |= !(isfinite(x) && isfinite(y) && isfinite(z));
    if ((double)j * h <= t_end) m0 = max(m0, __float_as_uint((float)sqrt(x * x + y * y + z * z)));
    if (j < N - 1) {
      const double* b = a + 3 * (j + 1);
      const double vx = (b[0] - x) / h, vy = (b[1] - y) / h, vz = (b[2] - z) / h;
      m2 = max(m2, __float_as_uint((float)sqrt(vx * vx + vy * vy + vz * vz)));
      if (j > 0) {
        const double* o = a + 3 * (j - 1);
        const double ux = vx - (x - o[0]) / h, uy = vy - (y - o[1]) / h, uz = vz - (z - o[2]) / h;
        m1 = max(m1, __float_as_uint((float)sqrt(ux * ux + uy * uy + uz * uz)));
      }
    }
  }
  if (threadIdx.x == 0) {
    // the displacement at t_end, on the segment that holds it (or the last one)
    const int j = (int)fmin((double)(N - 2), fmax(0.0, floor(t_end / h)));
    const double f = t_end / h - (double)j;
    double d2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double v = a[3 * j + k] + f * (a[3 * (j + 1) + k] - a[3 * j + k]);
      d2 += v * v;
    }
    m0 = max(m0, __float_as_uint((float)sqrt(d2)));
    bad |= !isfinite(d2);
  }
  atomicMax(&s_max[0], m0);
  atomicMax(&s_max[1], m1);
  atomicMax(&s_max[2], m2);
  if (bad) atomicOr(&s_max[3], 1u);
  __syncthreads();
  if (threadIdx.x == 0) {
    // maxima rounded to FP32: nudged up so that they stay bounds
    sw.tstats[p] = make_float4(__uint_as_float(s_max[0]) * 1.000001f, __uint_as_float(s_max[1]) * 1.000001f,
                               __uint_as_float(s_max[2]) * 1.000001f, s_max[3] ? 1.0f : 0.0f);
  }
}

// XCD queue of tile t: its swath's along-track stripe (eight stripes of
// whole tiles), rotated by the swath index so that small swaths of a batch
// spread over the dies.
__device__ __forceinline__ int tile_xcd(const Workspace& ws, int t) {
  const int s = ws.tile_swath[t];
  const SwathDev& sw = ws.swaths[s];
  const int tix = (t - sw.tile0) % sw.ntx;
  return (int)(((long long)tix * kXcds / sw.ntx + s) % kXcds);
}

// Single-workgroup counting sort of the tiles by XCD queue, then by cost
// bucket, largest first (longest-processing-time order within each queue);
// writes each queue's first slot and length. A stripe's tiles read the echo
// windows of the pings whose beams cover it, so its XCD's L2 serves them
// again; every stripe holds every range, so each queue ends on its cheapest
// tiles. Measured on the operational swath against one global LPT queue:
// 27% less HBM traffic and 1% less time; queues of equal-cost range bands
// cut the traffic by 35% but cost 4% more time (each die's tail is then made
// of its band's large tiles). The order inside a bucket depends on atomics;
// it affects only scheduling, never a pixel.
__device__ __forceinline__ int tile_bucket(const Workspace& ws, int t, int bucket_shift) {
  const PingRange pr = ws.prange[t];
  const long long npe = (pr.hi >= pr.lo) ? (long long)(pr.hi - pr.lo + 1) * ws.swaths[ws.tile_swath[t]].E : 0;
  const int b = (int)(npe >> bucket_shift);
  return b > kBuckets - 1 ? kBuckets - 1 : b;
}

__global__ __launch_bounds__(kThreads) void order_kernel(Workspace ws, int n_tiles, int bucket_shift) {
  __shared__ unsigned cursor[kXcds][kBuckets];
  for (int i = threadIdx.x; i < kXcds * kBuckets; i += blockDim.x) cursor[i / kBuckets][i % kBuckets] = 0u;
  __syncthreads();
  for (int t = threadIdx.x; t < n_tiles; t += blockDim.x)
    atomicAdd(&cursor[tile_xcd(ws, t)][tile_bucket(ws, t, bucket_shift)], 1u);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned run = 0;
    for (int x = 0; x < kXcds; ++x) {
      const unsigned start = run;
      for (int b = kBuckets - 1; b >= 0; --b) {
        const unsigned n = cursor[x][b];
        cursor[x][b] = run;
        run += n;
      }
      ws.counters[kQueueStart + x] = start;
      ws.counters[kQueueLen + x] = run - start;
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < n_tiles; t += blockDim.x) {
    const unsigned slot = atomicAdd(&cursor[tile_xcd(ws, t)][tile_bucket(ws, t, bucket_shift)], 1u);
    ws.order[slot] = t;
  }
}

// Continuous motion: per-record constants of the per-pixel correction, the
// receivers on the line R + q + v t.
//   hx = (C - R)_x, avyz = ((C - R)_y + dy) v_y + ((C - R)_z + dz) v_z for the
//   lane's row, (vx, vv) = (v_x, |v|^2), tc = (d0_T + d0_R + dc) / c with dc
//   the motion path at the tile centre, ic = 1 / c; for a position table also
//   (qx, aqyz) as (vx, avyz) for q, qq = |q|^2, qv = q.v.
struct MotionTerm {
  float hx, avyz, vx, vv, tc, dc, ic;
  float qx, aqyz, qq, qv;
};

// One (ping, element) record applied to the K pixels of a lane. DEG selects
// the receiver-leg offset (0 the exact form, 4 or 5 the series of that
// degree), TEST the per-pixel gate test of a partially gated record; both are
// uniform over the workgroup.
//
// MOT adds the receiver's motion during reception. With a = p - R (ping-time
// receiver), D the stop-and-hop path offset and tau_1 = tc + D / c (the
// pixel's delay with the centre's motion path dc), the motion path
// delta = |a - v tau| - |a| solves delta = f(delta); one Newton step from dc,
//     g = n / (|a - v tau_1| + |a|),  n = tau_1 (tau_1 |v|^2 - 2 a.v),
//     F = g - dc,  eps = (a.v - tau_1 |v|^2) / (c |a - v tau_1|),
//     delta = dc + F (1 - eps)
// TRK (a position table) replaces the displacement v tau by the line's
// w = q + v tau: n = |w|^2 - 2 a.w with a.w = a.q + tau_1 a.v and
// |w|^2 = |q|^2 + tau_1 (2 q.v + tau_1 |v|^2), eps = (a.v - w.v) / (c |a - w|).
// (the cancellation-free form of |a - w| - |a|; 1/(1 + eps) to first order,
// eps ~ |v|/c, and 1/|a - v tau_1| as 2 / (|a - v tau_1| + |a|); the step
// leaves errors far below a micrometre while |F| stays within the sample the
// plan allows). The record's reference already holds dc, so the offset grows
// by F (1 - eps).
template <int K, int LX, int DEG, bool TEST, bool MOT = false, bool TRK = false>
__device__ __forceinline__ void accumulate(const RxRec& rec, const float4* __restrict__ win, const float* dx,
                                           const float* dsq, const float* dT, float dyl, float dzl, float fs_c,
                                           float fc_c, float szero, int da, int span, float* accr,
                                           float* acci, const MotionTerm& mt = MotionTerm{}) {
  const float ryz = fmaf(rec.q0.y, dyl, rec.q0.z * dzl);
  const float d0 = rec.q1.w;
  const float d0sq = d0 * d0;
  // phase 1: delays, sample positions and carrier phases of the K pixels
  float sidx[K], cyc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const float num = fmaf(rec.q0.x, dx[k], ryz + dsq[k]);
    float D;   // two-way path offset from the (tile, ping, element) reference, metres
    if constexpr (MOT) {
      float dR;
      if (DEG > 0) {
        float h = DEG == 5 ? fmaf(rec.q1.z, num, rec.q2.w) : rec.q2.w;
        h = fmaf(h, num, rec.q2.z);
        h = fmaf(h, num, rec.q2.y);
        h = fmaf(h, num, rec.q2.x);
        dR = h * num;
      } else {
        const float sq = __builtin_amdgcn_sqrtf(d0sq + num);
        dR = num * __builtin_amdgcn_rcpf(d0 + sq);
      }
      D = dR + dT[k];
      const float hxd = mt.hx + dx[k];
      const float av = fmaf(hxd, mt.vx, mt.avyz);
      const float am = d0 + dR;
      const float t1 = fmaf(D, mt.ic, mt.tc);
      float n, wv;
      if constexpr (TRK) {
        const float aq = fmaf(hxd, mt.qx, mt.aqyz);
        const float ww = fmaf(t1, fmaf(t1, mt.vv, 2.0f * mt.qv), mt.qq);
        n = fmaf(-2.0f, fmaf(t1, av, aq), ww);
        wv = fmaf(t1, mt.vv, mt.qv);
      } else {
        wv = t1 * mt.vv;
        n = t1 * fmaf(-2.0f, av, wv);
      }
      const float rr = __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(fmaf(am, am, n)) + am);
      const float F = fmaf(n, rr, -mt.dc);
      const float eps = (av - wv) * (2.0f * mt.ic * rr);
      D += fmaf(-F, eps, F);
    } else if (DEG > 0) {
      float h = DEG == 5 ? fmaf(rec.q1.z, num, rec.q2.w) : rec.q2.w;
      h = fmaf(h, num, rec.q2.z);
      h = fmaf(h, num, rec.q2.y);
      h = fmaf(h, num, rec.q2.x);
      D = fmaf(h, num, dT[k]);
    } else {
      const float sq = __builtin_amdgcn_sqrtf(d0sq + num);
      D = fmaf(num, __builtin_amdgcn_rcpf(d0 + sq), dT[k]);
    }
    float si = fmaf(D, fs_c, rec.q1.x);   // sample position - 1/2 in the window
    cyc[k] = fmaf(D, fc_c, rec.q1.y);     // the hardware sin/cos take revolutions
    if (TEST) {
      const bool in = (unsigned)(da + LX * k) <= (unsigned)span;
      si = in ? si : szero;
    }
    sidx[k] = si;
  }
  // phase 2: every window read in flight at once
  float4 v[K];
  float wt[K];
  const unsigned wbase = window_base(win);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = window_read(wbase, sidx[k], &wt[k]);
  // phase 3: carrier phasors while the reads land
  float sn[K], cs[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    sn[k] = __builtin_amdgcn_sinf(cyc[k]);
    cs[k] = __builtin_amdgcn_cosf(cyc[k]);
  }
  // phase 4: interpolate and accumulate
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const float vr = fmaf(wt[k], v[k].z, v[k].x);
    const float vi = fmaf(wt[k], v[k].w, v[k].y);
    accr[k] = fmaf(vr, cs[k], accr[k]);
    accr[k] = fmaf(-vi, sn[k], accr[k]);
    acci[k] = fmaf(vr, sn[k], acci[k]);
    acci[k] = fmaf(vi, cs[k], acci[k]);
  }
}

// sin(pi x) / pi for x in [0, 1], accurate relative to its value (the
// hardware sine is accurate only in absolute terms, which is too coarse near
// x = 0 and x = 1, where the central sinc tap divides by a small distance):
// by symmetry x -> min(x, 1 - x) in [0, 1/2], then the Taylor series of
// sin(pi x) / pi through x^11 (truncation below 6e-8 relative at x = 1/2).
__device__ __forceinline__ float sin_pi_over_pi(float x) {
  const float y = fminf(x, 1.0f - x);
  const float y2 = y * y;
  const float p2 = 9.8696044010893586f;   // pi^2
  float h = -p2 / 39916800.0f * p2 * p2 * p2 * p2;   // -pi^10 / 11!
  h = fmaf(h, y2, p2 * p2 * p2 * p2 / 362880.0f);    // +pi^8 / 9!
  h = fmaf(h, y2, -p2 * p2 * p2 / 5040.0f);          // -pi^6 / 7!
  h = fmaf(h, y2, p2 * p2 / 120.0f);                 // +pi^4 / 5!
  h = fmaf(h, y2, -p2 / 6.0f);                       // -pi^2 / 3!
  h = fmaf(h, y2, 1.0f);
  return y * h;
}

// The windowed-sinc variant of accumulate(): L = sum over the 8 samples m
// around u of E~[m] h(u - m), h(t) = sinc(t) (1 + cos(pi t / 4)) / 2. With
// n = floor(s) and w = s - n (s the sample position in the window), tap j
// (j = 0..7, sample n - 3 + j) is at t_j = w + 3 - j, and
//   sinc(t_j) = (-1)^(3-j) sin(pi w) / (pi t_j),
//   cos(pi t_j / 4) = cos(th) cos(j pi / 4) + sin(th) sin(j pi / 4), th = pi (w + 3) / 4,
// so one sine, one sine/cosine pair and eight reciprocals serve the 8 taps.
// w is kept in [1e-6, 1 - 1e-6] so that no t_j is zero (an offset of at most
// 1e-6 samples). Gated-out pixels read samples 0..8 and are weighted by zero.
template <int K, int LX, int DEG, bool TEST>
__device__ __forceinline__ void accumulate_sinc(const RxRec& rec, const float2* __restrict__ win, const float* dx,
                                                const float* dsq, const float* dT, float dyl, float dzl, float fs_c,
                                                float fc_c, int da, int span, float* accr, float* acci) {
  const float ryz = fmaf(rec.q0.y, dyl, rec.q0.z * dzl);
  const float d0 = rec.q1.w;
  const float d0sq = d0 * d0;
  const unsigned wbase = lds_address(win) + 8u - (kRoundMagicBits << 3);   // entry of sample n - 3 is n + 1
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const float num = fmaf(rec.q0.x, dx[k], ryz + dsq[k]);
    float D;
    if (DEG > 0) {
      float h = DEG == 5 ? fmaf(rec.q1.z, num, rec.q2.w) : rec.q2.w;
      h = fmaf(h, num, rec.q2.z);
      h = fmaf(h, num, rec.q2.y);
      h = fmaf(h, num, rec.q2.x);
      D = fmaf(h, num, dT[k]);
    } else {
      const float sq = __builtin_amdgcn_sqrtf(d0sq + num);
      D = fmaf(num, __builtin_amdgcn_rcpf(d0 + sq), dT[k]);
    }
    float sh = fmaf(D, fs_c, rec.q1.x);   // s - 1/2
    const float cyc = fmaf(D, fc_c, rec.q1.y);
    float keep = 1.0f;
    if (TEST) {
      const bool in = (unsigned)(da + LX * k) <= (unsigned)span;
      sh = in ? sh : 0.0f;
      keep = in ? 1.0f : 0.0f;
    }
    const float t = sh + kRoundMagic;                 // n = round(s - 1/2) = floor(s)
    const float w = fminf(fmaxf(sh - (t - kRoundMagic) + 0.5f, 1e-6f), 1.0f - 1e-6f);
    const unsigned addr = wbase + (__float_as_uint(t) << 3);
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    const __attribute__((address_space(3))) f32x2* e =
        reinterpret_cast<const __attribute__((address_space(3))) f32x2*>((uintptr_t)addr);
    const float a = keep * sin_pi_over_pi(w) * 0.5f;  // sin(pi w) / pi, times the window's 1/2
    const float th = (w + 3.0f) * 0.125f;             // revolutions: pi (w + 3) / 4
    const float cth = __builtin_amdgcn_cosf(th), sth = __builtin_amdgcn_sinf(th);
    float lr = 0.0f, li = 0.0f;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      constexpr float kC[8] = {1.0f, 0.70710678f, 0.0f, -0.70710678f, -1.0f, -0.70710678f, 0.0f, 0.70710678f};
      constexpr float kS[8] = {0.0f, 0.70710678f, 1.0f, 0.70710678f, 0.0f, -0.70710678f, -1.0f, -0.70710678f};
      const float tj = w + (float)(3 - j);
      const float hann2 = fmaf(cth, kC[j], fmaf(sth, kS[j], 1.0f));   // 1 + cos(pi t_j / 4)
      const float sg = ((3 - j) & 1) ? -a : a;                        // (-1)^(3-j) sin(pi w) / (2 pi)
      const float hw = sg * __builtin_amdgcn_rcpf(tj) * hann2;
      const f32x2 v = e[j];
      lr = fmaf(hw, v.x, lr);
      li = fmaf(hw, v.y, li);
    }
    const float sn = __builtin_amdgcn_sinf(cyc);
    const float cs = __builtin_amdgcn_cosf(cyc);
    accr[k] = fmaf(lr, cs, accr[k]);
    accr[k] = fmaf(-li, sn, accr[k]);
    acci[k] = fmaf(lr, sn, acci[k]);
    acci[k] = fmaf(li, cs, acci[k]);
  }
}

// The read-only tables are separate restrict-qualified arguments so that the
// compiler may read them through the scalar cache.
template <int L, bool GATE, int DT, int INTERP>
__global__ __launch_bounds__(kLayouts[L].LX * kLayouts[L].LY * kLayouts[L].LZ)
__attribute__((amdgpu_waves_per_eu(kImageWaves, kImageWaves))) void image_kernel(
    Workspace ws, const SwathDev* __restrict__ swaths, const int* __restrict__ order,
    const int* __restrict__ tile_swath, const PingRange* __restrict__ prange, int n_tiles) {
  extern __shared__ __align__(16) unsigned char lds[];
  constexpr int K = kLayouts[L].K, LX = kLayouts[L].LX, LY = kLayouts[L].LY, LZ = kLayouts[L].LZ;
  constexpr int NT = LX * LY * LZ;
  constexpr int TX = LX * K, TY = LY, TZ = LZ, ROWS = LY * LZ;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lx = tid % LX, ly = (tid / LX) % LY, lz = tid / (LX * LY);
  const int row = ly + LY * lz;
  __shared__ int s_item;
  __shared__ int s_npart;
  const int xcd = blockIdx.x % kXcds;

  for (;;) {
    __syncthreads();
    if (tid == 0) s_item = next_tile(ws, xcd);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);
    if (item < 0) break;
    const int t = __builtin_amdgcn_readfirstlane(order[item]);
    const int s = __builtin_amdgcn_readfirstlane(tile_swath[t]);
    const SwathDev& sw = swaths[s];
    const int E = sw.E, W = sw.W, RC = sw.RC;
    const int lt = t - sw.tile0;
    const int tix = lt % sw.ntx, tiy = (lt / sw.ntx) % sw.nty, tiz = lt / (sw.ntx * sw.nty);
    const int x0 = tix * TX, y0 = tiy * TY, z0 = tiz * TZ;
    double C[3];
    C[0] = tile_centre(sw, 0, x0, TX);
    C[1] = tile_centre(sw, 1, y0, TY);
    C[2] = tile_centre(sw, 2, z0, TZ);
    const double c = *sw.c;
    const float fs_c = (float)(sw.fs / c);
    const float fc_c = (float)(sw.fc / c);
    const float ic = (float)(1.0 / c);
    const PingRange pr = prange[t];
    constexpr bool MOT = INTERP >= 2;   // linear interpolation, receivers moving during reception
    constexpr bool TRK = INTERP == 3;   // ... along a position table
    const LdsLayout Ld = lds_layout(RC, chunk_pings(RC, E), W, ROWS, GATE, MOT);
    const TxRec* ltx = reinterpret_cast<const TxRec*>(lds + Ld.off_tx);
    const RxRec* lrx = reinterpret_cast<const RxRec*>(lds + Ld.off_rx);
    const int* lrows = reinterpret_cast<const int*>(lds + Ld.off_rows);
    const float4* lwin = reinterpret_cast<const float4*>(lds + Ld.off_win);

    // per-lane pixel offsets from the tile centre (exact multiples of the spacing)
    const float sx = (float)sw.d[0], sy = (float)sw.d[1], sz = (float)sw.d[2];
    float dx[K], dsq[K];
    const float dyl = (float)(2 * ly - (TY - 1)) * 0.5f * sy;
    const float dzl = (float)(2 * lz - (TZ - 1)) * 0.5f * sz;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      dx[k] = (float)(2 * (lx + LX * k) - (TX - 1)) * 0.5f * sx;
      dsq[k] = dx[k] * dx[k] + dyl * dyl + dzl * dzl;
    }
    float accr[K], acci[K];
#pragma unroll
    for (int k = 0; k < K; ++k) { accr[k] = 0.0f; acci[k] = 0.0f; }
    const float szero = (float)W;   // the window's all-zero entry

    const Geo geo = geo_for(ws, sw, ROWS, GATE);
    int* lpart = reinterpret_cast<int*>(lds + Ld.off_win);   // window area, free between chunks

    for (int P0 = pr.lo; P0 <= pr.hi; P0 += sw.SC) {
      const int sc = min(sw.SC, pr.hi - P0 + 1);
      __syncthreads();
      build_geometry<NT, TX, LY, LZ, GATE, MOT>(geo, lpart, &s_npart, ws, sw, c, C, P0, sc, x0, y0, z0, tid);
      // chunks of RC records (ping-major) of the run; a chunk may hold part
      // of a ping, a whole ping or several pings. The transmitter leg dT of
      // a ping split over two chunks is formed once.
      float dT[K];
      int dT_slot = -1;
      float d0T = 0.0f;
      float4 vel = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      float4 line_q = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      float line_qv = 0.0f;
      for (int q0 = 0; q0 < sc * E; q0 += RC) {
        const int nr = min(RC, sc * E - q0);
        const int sa = q0 / E, sb = (q0 + nr - 1) / E;
        if (q0 > 0) __syncthreads();
        // staging rows per wave: four for the 3D tiles' 32-record chunks
        // (399 ms against 405 ms with three on the 3D volume)
        load_chunk<NT, ROWS, GATE, DT, INTERP == 1, MOT, (LZ > 1 ? 4 : 3)>(lds, geo, sw, P0, q0, nr, sa,
                                                                           sb - sa + 1, Ld, tid, lane, wave);
        for (int slot = sa; slot <= sb; ++slot) {
          if (slot != dT_slot) {
            const TxRec tr = ltx[slot - sa];
            const float tyz = fmaf(tr.uy2, dyl, tr.uz2 * dzl);
#pragma unroll
            for (int k = 0; k < K; ++k) {
              const float num = fmaf(tr.ux2, dx[k], tyz + dsq[k]);
              const float sq = __builtin_amdgcn_sqrtf(tr.d0sq + num);
              dT[k] = num * __builtin_amdgcn_rcpf(tr.d0 + sq);
            }
            dT_slot = slot;
            if (MOT) {
              d0T = tr.d0;
              const float4* lline = reinterpret_cast<const float4*>(lds + Ld.off_vel) + 3 * (slot - sa);
              vel = lline[0];
              if (TRK) {
                line_q = lline[1];
                line_qv = lline[2].x;
              }
            }
          }
          const int r_lo = max(slot * E, q0) - q0, r_hi = min(slot * E + E, q0 + nr) - q0;
          for (int r = r_lo; r < r_hi; ++r) {
            const unsigned f = __builtin_amdgcn_readfirstlane(__float_as_uint(lrx[r].q0.w));
            if (f & kFlagSkip) continue;
            const RxRec rec = lrx[r];
            const float4* win = lwin + (size_t)r * (W + 1);
            if (INTERP == 1) {
              const float2* rwin = reinterpret_cast<const float2*>(win);
              int da = 0, span = 0;
              if (GATE && !(f & kFlagFull)) {
                const int v = lrows[r * ROWS + row];
                da = lx - row_lo(v);
                span = row_hi(v) - row_lo(v);
              }
              const bool test = GATE && !(f & kFlagFull);
              if (f & kFlagPoly) {
                if (test) accumulate_sinc<K, LX, 5, true>(rec, rwin, dx, dsq, dT, dyl, dzl, fs_c, fc_c, da, span, accr, acci);
                else accumulate_sinc<K, LX, 5, false>(rec, rwin, dx, dsq, dT, dyl, dzl, fs_c, fc_c, 0, 0, accr, acci);
              } else {
                if (test) accumulate_sinc<K, LX, 0, true>(rec, rwin, dx, dsq, dT, dyl, dzl, fs_c, fc_c, da, span, accr, acci);
                else accumulate_sinc<K, LX, 0, false>(rec, rwin, dx, dsq, dT, dyl, dzl, fs_c, fc_c, 0, 0, accr, acci);
              }
              continue;
            }
            if constexpr (MOT) {
              MotionTerm mt;
              mt.hx = 0.5f * rec.q0.x;
              mt.avyz = fmaf(fmaf(0.5f, rec.q0.y, dyl), vel.y, fmaf(0.5f, rec.q0.z, dzl) * vel.z);
              mt.vx = vel.x;
              mt.vv = vel.w;
              if (TRK) {
                mt.qx = line_q.x;
                mt.aqyz = fmaf(fmaf(0.5f, rec.q0.y, dyl), line_q.y, fmaf(0.5f, rec.q0.z, dzl) * line_q.z);
                mt.qq = line_q.w;
                mt.qv = line_qv;
              }
              mt.ic = ic;
              mt.dc = reinterpret_cast<const float*>(lds + Ld.off_dc)[r];
              mt.tc = (d0T + rec.q1.w + mt.dc) * ic;
              int da = 0, span = 0;
              const bool test = GATE && !(f & kFlagFull);
              if (test) {
                const int v = lrows[r * ROWS + row];
                da = lx - row_lo(v);
                span = row_hi(v) - row_lo(v);
              }
              if (f & kFlagPoly) {
                if (test) accumulate<K, LX, 5, true, true, TRK>(rec, win, dx, dsq, dT, dyl, dzl, fs_c, fc_c, szero, da, span, accr, acci, mt);
                else accumulate<K, LX, 5, false, true, TRK>(rec, win, dx, dsq, dT, dyl, dzl, fs_c, fc_c, szero, 0, 0, accr, acci, mt);
              } else {
                if (test) accumulate<K, LX, 0, true, true, TRK>(rec, win, dx, dsq, dT, dyl, dzl, fs_c, fc_c, szero, da, span, accr, acci, mt);
                else accumulate<K, LX, 0, false, true, TRK>(rec, win, dx, dsq, dT, dyl, dzl, fs_c, fc_c, szero, 0, 0, accr, acci, mt);
              }
              continue;
            }
            if (!GATE || (f & kFlagFull)) {
              if (f & kFlagDeg4)
                accumulate<K, LX, 4, false>(rec, win, dx, dsq, dT, dyl, dzl, fs_c, fc_c, szero, 0, 0, accr, acci);
              else if (f & kFlagPoly)
                accumulate<K, LX, 5, false>(rec, win, dx, dsq, dT, dyl, dzl, fs_c, fc_c, szero, 0, 0, accr, acci);
              else
                accumulate<K, LX, 0, false>(rec, win, dx, dsq, dT, dyl, dzl, fs_c, fc_c, szero, 0, 0, accr, acci);
            } else {
              const int v = lrows[r * ROWS + row];
              const int a = row_lo(v), b = row_hi(v);
              if (f & kFlagDeg4)
                accumulate<K, LX, 4, true>(rec, win, dx, dsq, dT, dyl, dzl, fs_c, fc_c, szero, lx - a, b - a, accr,
                                           acci);
              else if (f & kFlagPoly)
                accumulate<K, LX, 5, true>(rec, win, dx, dsq, dT, dyl, dzl, fs_c, fc_c, szero, lx - a, b - a, accr,
                                           acci);
              else
                accumulate<K, LX, 0, true>(rec, win, dx, dsq, dT, dyl, dzl, fs_c, fc_c, szero, lx - a, b - a, accr,
                                           acci);
            }
          }
        }
      }
    }
    // write the tile once
    const int iy = y0 + ly, iz = z0 + lz;
    if (iy < sw.ny && iz < sw.nz) {
      float2* out = sw.image + ((size_t)iz * sw.ny + iy) * (size_t)sw.nx;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int ix = x0 + lx + LX * k;
        if (ix < sw.nx) out[ix] = make_float2(accr[k], acci[k]);
      }
    }
  }
}

// ------------------------------------------------------------ dispatch ---

typedef void (*ImageKernelFn)(Workspace, const SwathDev*, const int*, const int*, const PingRange*, int);

template <int L, int INTERP>
static ImageKernelFn image_for_layout(bool gate, int dt) {
  if (gate) {
    switch (dt) {
      case 0: return image_kernel<L, true, 0, INTERP>;
      case 1: return image_kernel<L, true, 1, INTERP>;
      default: return image_kernel<L, true, 2, INTERP>;
    }
  }
  switch (dt) {
    case 0: return image_kernel<L, false, 0, INTERP>;
    case 1: return image_kernel<L, false, 1, INTERP>;
    default: return image_kernel<L, false, 2, INTERP>;
  }
}

template <int INTERP>
static ImageKernelFn image_for_interp(int layout, bool gate, int dt) {
  switch (layout) {
    case 0: return image_for_layout<0, INTERP>(gate, dt);
    case 1: return image_for_layout<1, INTERP>(gate, dt);
    case 2: return image_for_layout<2, INTERP>(gate, dt);
    case 3: return image_for_layout<3, INTERP>(gate, dt);
    case 4: return image_for_layout<4, INTERP>(gate, dt);
    case 5: return image_for_layout<5, INTERP>(gate, dt);
    case 6: return image_for_layout<6, INTERP>(gate, dt);
    case 7: return image_for_layout<7, INTERP>(gate, dt);
    case 8: return image_for_layout<8, INTERP>(gate, dt);
    default: return nullptr;
  }
}

// interp: 0 linear, 1 windowed sinc, 2 linear with the receivers moving during
// reception at a velocity, 3 ... along a position table
ImageKernelFn image_kernel_for(int layout, bool gate, int dt, int interp) {
  switch (interp) {
    case 1: return image_for_interp<1>(layout, gate, dt);
    case 2: return image_for_interp<2>(layout, gate, dt);
    case 3: return image_for_interp<3>(layout, gate, dt);
    default: return image_for_interp<0>(layout, gate, dt);
  }
}

int image_lds_bytes(int RC, int E, int W, int ROWS, bool gate, bool motion) {
  return lds_layout(RC, chunk_pings(RC, E), W, ROWS, gate, motion).bytes;
}

hipError_t launch_init(const Workspace& ws, hipStream_t st) {
  hipLaunchKernelGGL(init_kernel, dim3(1), dim3(64), 0, st, ws);
  return hipGetLastError();
}

hipError_t launch_cull(const Workspace& ws, int n_tiles, int TX, int TY, int TZ, int bucket_shift,
                       hipStream_t st) {
  hipLaunchKernelGGL(cull_kernel, dim3(n_tiles), dim3(kThreads), 0, st, ws, TX, TY, TZ, bucket_shift);
  return hipGetLastError();
}

hipError_t launch_track_stats(const Workspace& ws, int swath, int n_ping, hipStream_t st) {
  hipLaunchKernelGGL(track_stats_kernel, dim3(n_ping), dim3(kThreads), 0, st, ws, swath);
  return hipGetLastError();
}

hipError_t launch_order(const Workspace& ws, int n_tiles, int bucket_shift, hipStream_t st) {
  hipLaunchKernelGGL(order_kernel, dim3(1), dim3(kThreads), 0, st, ws, n_tiles, bucket_shift);
  return hipGetLastError();
}

hipError_t launch_image(ImageKernelFn fn, const Workspace& ws, int n_tiles, int grid, int threads, int lds_bytes,
                        hipStream_t st) {
  hipLaunchKernelGGL(fn, dim3(grid), dim3(threads), lds_bytes, st, ws, (const SwathDev*)ws.swaths,
                     (const int*)ws.order, (const int*)ws.tile_swath, (const PingRange*)ws.prange, n_tiles);
  return hipGetLastError();
}

hipError_t image_occupancy(ImageKernelFn fn, int threads, int lds_bytes, int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, threads, lds_bytes);
}

hipError_t set_image_lds_limit(ImageKernelFn fn, int lds_bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                             lds_bytes);
}

}  // namespace sasbp

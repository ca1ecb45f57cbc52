// Device-side pieces shared by the image and adjoint kernels: the FP64
// reference geometry of a (tile, ping, element), the exact per-row beam-gate
// intervals, and the staging of echo windows into LDS.
//
// Delay model (Eq. 1, Sec. II-A): tau = (|p - T| + |p - R|) / c. Inside a tile
// with centre C, a pixel is p = C + delta. With u = C - X for an apex X (the
// transmitter or a receiver) and d0 = |u|,
//     |p - X| - d0 = num / (d0 + sqrt(d0^2 + num)),   num = 2 u.delta + |delta|^2,
// which has no cancellation, so the offset is accurate in FP32 while C, d0,
// the reference delay and its carrier phase are formed in FP64. Absolute
// ranges of tens of metres against a 1.5 cm wavelength would lose the phase in
// FP32.
#pragma once

#include "tdbp_dev.h"

namespace sasbp {

// One receiver record per (ping, element), 8 floats = 32 bytes:
//   [0..2] 2 u_R (x, y, z)   [3] d0_R   [4] d0_R^2
//   [5] s0: reference delay in samples relative to the window start
//   [6] phi0: frac(f_c * tau_ref), cycles
//   [7] flags (bit pattern): 1 = no pixel of the tile is gated in, 2 = every pixel is
struct RxRec {
  float ux2, uy2, uz2, d0, d0sq, s0, phi0, flags;
};
// One transmitter record per ping.
struct TxRec {
  float ux2, uy2, uz2, d0, d0sq, pad0, pad1, pad2;
};

constexpr unsigned kFlagSkip = 1u;
constexpr unsigned kFlagFull = 2u;
constexpr int kEmptyRow = 30000;   // encodes an empty gate interval (never matches a local x)

__device__ __forceinline__ double tile_centre(const SwathDev& sw, int a, int first, int extent) {
  return sw.o[a] + ((double)first + 0.5 * (double)(extent - 1)) * sw.d[a];
}

__device__ __forceinline__ bool finite3(double a, double b, double c) {
  return isfinite(a) && isfinite(b) && isfinite(c);
}

// Receiver record and window start for (ping p, element e) of the tile centred at C.
// Returns false if the navigation is not finite.
__device__ __forceinline__ bool make_rx_record(const SwathDev& sw, double c, const double C[3], int p, int e,
                                               RxRec* rec, int* n0_out) {
  const double* T = sw.tx + (size_t)p * 3;
  const double* R = sw.rx + ((size_t)p * sw.E + e) * 3;
  const double tx0 = T[0], tx1 = T[1], tx2 = T[2];
  const double rx0 = R[0], rx1 = R[1], rx2 = R[2];
  const double uT0 = C[0] - tx0, uT1 = C[1] - tx1, uT2 = C[2] - tx2;
  const double uR0 = C[0] - rx0, uR1 = C[1] - rx1, uR2 = C[2] - rx2;
  const double d0T = sqrt(uT0 * uT0 + uT1 * uT1 + uT2 * uT2);
  const double d0R = sqrt(uR0 * uR0 + uR1 * uR1 + uR2 * uR2);
  const bool ok = finite3(tx0, tx1, tx2) && finite3(rx0, rx1, rx2);
  const double tau = (d0T + d0R) / c;
  const double uref = (tau - sw.t0) * sw.fs;
  const double span = 2.0 * sw.half_diag * sw.fs / c;
  double nstart = floor(uref - span) - 2.0;
  if (!(nstart > -1.0e9)) nstart = -1.0e9;          // also maps NaN to a harmless value
  if (nstart > 1.0e9) nstart = 1.0e9;
  const int n0 = (int)nstart;
  const double cyc = sw.fc * tau;
  rec->ux2 = (float)(2.0 * uR0);
  rec->uy2 = (float)(2.0 * uR1);
  rec->uz2 = (float)(2.0 * uR2);
  rec->d0 = (float)d0R;
  rec->d0sq = (float)(d0R * d0R);
  rec->s0 = (float)(uref - (double)n0);
  rec->phi0 = (float)(cyc - floor(cyc));
  rec->flags = __uint_as_float(ok ? 0u : kFlagSkip);
  *n0_out = n0;
  return ok;
}

__device__ __forceinline__ void make_tx_record(const SwathDev& sw, const double C[3], int p, TxRec* rec) {
  const double* T = sw.tx + (size_t)p * 3;
  const double u0 = C[0] - T[0], u1 = C[1] - T[1], u2 = C[2] - T[2];
  const double d0 = sqrt(u0 * u0 + u1 * u1 + u2 * u2);
  rec->ux2 = (float)(2.0 * u0);
  rec->uy2 = (float)(2.0 * u1);
  rec->uz2 = (float)(2.0 * u2);
  rec->d0 = (float)d0;
  rec->d0sq = (float)(d0 * d0);
  rec->pad0 = rec->pad1 = rec->pad2 = 0.0f;
}

// Exact gate interval of tile row (y, z) for (ping p, element e): local x indices
// [a, b] (relative to the tile's first x) whose pixels satisfy
// |x - T_x| <= tan(g) rho_T and |x - R_x| <= tan(g) rho_R, the per-row form of
// |dx| <= sin(g) |p - X| (rho = (y, z) distance to the apex). FP64.
__device__ __forceinline__ int gate_row(const SwathDev& sw, int p, int e, double y, double z, int x0, int TX) {
  const double* T = sw.tx + (size_t)p * 3;
  const double* R = sw.rx + ((size_t)p * sw.E + e) * 3;
  const double hT = sw.tan_g * sqrt((y - T[1]) * (y - T[1]) + (z - T[2]) * (z - T[2]));
  const double hR = sw.tan_g * sqrt((y - R[1]) * (y - R[1]) + (z - R[2]) * (z - R[2]));
  const double lo = fmax(T[0] - hT, R[0] - hR);
  const double hi = fmin(T[0] + hT, R[0] + hR);
  const double fa = ceil((lo - sw.o[0]) / sw.d[0]) - (double)x0;
  const double fb = floor((hi - sw.o[0]) / sw.d[0]) - (double)x0;
  // clamp to the tile (also maps NaN to an empty row)
  const double ca = fmax(fa, 0.0);
  const double cb = fmin(fb, (double)(TX - 1));
  if (!(ca <= cb)) return (kEmptyRow & 0xffff) | (kEmptyRow << 16);
  const int a = (int)ca, b = (int)cb;
  return (a & 0xffff) | (b << 16);
}

__device__ __forceinline__ int row_lo(int v) { return (int)(short)(v & 0xffff); }
__device__ __forceinline__ int row_hi(int v) { return v >> 16; }

// Echo sample loaders: FP32 complex out of each storage type.
__device__ __forceinline__ float2 load_sample(const void* base, size_t idx, int dtype, float scale) {
  if (dtype == 0) {
    return reinterpret_cast<const float2*>(base)[idx];
  } else if (dtype == 1) {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    const h2 v = reinterpret_cast<const h2*>(base)[idx];
    return make_float2((float)v.x * scale, (float)v.y * scale);
  } else {
    const unsigned v = reinterpret_cast<const unsigned*>(base)[idx];
    return make_float2(__uint_as_float(v << 16) * scale, __uint_as_float(v & 0xffff0000u) * scale);
  }
}

// LDS layout for a chunk of CP pings with E elements and window length W:
//   TxRec  tx[CP]            RxRec rx[CP][E]          int n0[CP][E]
//   int    rows[CP][E][ROWS] (gate only)              float2 win[CP][E][W+2]
struct LdsLayout {
  int off_tx, off_rx, off_n0, off_rows, off_win, bytes;
};

__host__ __device__ inline LdsLayout lds_layout(int CP, int E, int W, int ROWS, bool gate) {
  LdsLayout L;
  int o = 0;
  L.off_tx = o;   o += CP * (int)sizeof(TxRec);
  L.off_rx = o;   o += CP * E * (int)sizeof(RxRec);
  L.off_n0 = o;   o += CP * E * 4;
  L.off_rows = o; o += gate ? CP * E * ROWS * 4 : 0;
  o = (o + 15) & ~15;
  L.off_win = o;  o += CP * E * (W + 2) * 8;
  L.bytes = o;
  return L;
}

// Steps 1-2 of a chunk of pings, shared by the image and adjoint kernels:
// FP64 reference records, exact gate rows and (ping, element) flags, then the
// echo windows in LDS. Ends with a barrier; the caller must have passed a
// barrier since the previous chunk's last read of LDS.
template <int TX, int LY, int LZ, bool GATE, int DT>
__device__ __forceinline__ void prepare_chunk(unsigned char* lds, const Workspace& ws, const SwathDev& sw, double c,
                                              const double C[3], int p0, int cp, int x0, int y0, int z0,
                                              const LdsLayout& L, int tid, int lane, int wave) {
  constexpr int ROWS = LY * LZ;
  const int E = sw.E, W = sw.W;
  TxRec* ltx = reinterpret_cast<TxRec*>(lds + L.off_tx);
  RxRec* lrx = reinterpret_cast<RxRec*>(lds + L.off_rx);
  int* ln0 = reinterpret_cast<int*>(lds + L.off_n0);
  int* lrows = reinterpret_cast<int*>(lds + L.off_rows);
  float2* lwin = reinterpret_cast<float2*>(lds + L.off_win);
  // 1. FP64 reference geometry
  for (int r = tid; r < cp * E; r += kThreads) {
    const int slot = r / E, e = r - slot * E;
    RxRec rec;
    int n0;
    if (!make_rx_record(sw, c, C, p0 + slot, e, &rec, &n0)) atomicOr(&ws.counters[1], kStatusNav);
    lrx[r] = rec;
    ln0[r] = n0;
  }
  for (int r = tid; r < cp; r += kThreads) make_tx_record(sw, C, p0 + r, &ltx[r]);
  // a swath without a gate inside a plan whose kernel gates: every pixel is in
  const bool gate_on = GATE && sw.tan_g > 0.0;
  if (gate_on) {
    for (int q = tid; q < cp * E * ROWS; q += kThreads) {
      const int pe = q / ROWS, rr = q - pe * ROWS;
      const int slot = pe / E, e = pe - slot * E;
      const int ry = rr % LY, rz = rr / LY;
      const double y = sw.o[1] + (double)(y0 + ry) * sw.d[1];
      const double z = sw.o[2] + (double)(z0 + rz) * sw.d[2];
      lrows[q] = gate_row(sw, p0 + slot, e, y, z, x0, TX);
    }
  }
  __syncthreads();
  if (GATE && !gate_on) {
    for (int r = tid; r < cp * E; r += kThreads)
      lrx[r].flags = __uint_as_float(__float_as_uint(lrx[r].flags) | kFlagFull);
    __syncthreads();
  }
  if (gate_on) {
    // (ping, element) flags from the row intervals: skip / full tile
    for (int r = tid; r < cp * E; r += kThreads) {
      bool any = false, all = true;
      for (int rr = 0; rr < ROWS; ++rr) {
        const int v = lrows[r * ROWS + rr];
        const int a = row_lo(v), b = row_hi(v);
        const bool nonempty = a <= b;
        any |= nonempty;
        all &= nonempty && a == 0 && b == TX - 1;
      }
      unsigned f = __float_as_uint(lrx[r].flags);
      if (!any) f |= kFlagSkip;
      if (all) f |= kFlagFull;
      lrx[r].flags = __uint_as_float(f);
    }
    __syncthreads();
  }
  // 2. echo windows -> LDS
  for (int r = wave; r < cp * E; r += kThreads / 64) {
    const unsigned f = __float_as_uint(lrx[r].flags);
    if (f & kFlagSkip) continue;
    const int slot = r / E, e = r - slot * E;
    const int p = p0 + slot;
    const int n0 = ln0[r];
    const size_t rowbase = ((size_t)p * E + e) * (size_t)sw.Ns;
    const float scale = DT == 0 ? 1.0f : sw.scale[p];
    float2* dst = lwin + (size_t)r * (W + 2);
    for (int k = lane; k < W + 2; k += 64) {
      const int n = n0 + k;
      float2 v = make_float2(0.0f, 0.0f);
      if (k < W && n >= 0 && n < sw.Ns) v = load_sample(sw.echo, rowbase + (size_t)n, DT, scale);
      dst[k] = v;
    }
  }
  __syncthreads();
}

}  // namespace sasbp

// Device-side pieces shared by the image and adjoint kernels: the FP64
// reference geometry of a (tile, ping, element), the beam-gate classification
// and exact per-row gate intervals, and the staging of echo windows into LDS.
//
// Delay model (Eq. 1, Sec. II-A): tau = (|p - T| + |p - R|) / c. Inside a tile
// with centre C, a pixel is p = C + delta. With u = C - X for an apex X (the
// transmitter or a receiver), d0 = |u| and num = 2 u.delta + |delta|^2,
//     |p - X| - d0 = sqrt(d0^2 + num) - d0 = num / (d0 + sqrt(d0^2 + num)),
// a form without cancellation, so the offset is accurate in FP32 while C, d0,
// the reference delay and its carrier phase are formed in FP64 (absolute
// ranges of tens of metres against a 1.5 cm wavelength would lose the phase in
// FP32). For the receiver leg, evaluated once per (pixel, ping, element), the
// offset is the Taylor series of d0 (sqrt(1 + y) - 1), y = num / d0^2, in
// powers of num through num^5 whenever an FP64 bound on the truncation error
// over the whole tile is below 1e-8 m (0.004 mrad of two-way phase at 1.5 cm);
// otherwise the exact form above is used. The choice is per
// (tile, ping, element) and uniform across the workgroup.
#pragma once

#include "tdbp_dev.h"

namespace sasbp {

// Receiver record per (ping, element), 12 floats = three 16-byte LDS reads:
//   q0: 2 u_R (x, y, z), flags
//   q1: s0 - 1/2, s0 = reference delay in samples from the window start,
//       phi0 = frac(f_c tau_ref) in cycles, a5, d0_R
//   q2: a1..a4
// with Delta_R ~= num (a1 + num (a2 + num (a3 + num (a4 + num a5)))).
struct RxRec {
  float4 q0, q1, q2;
};
// Transmitter record per ping: 2 u_T (x, y, z), d0_T, d0_T^2, and the
// ping's dequantisation scale for 16-bit echo storage (1 for FP32).
struct TxRec {
  float ux2, uy2, uz2, d0, d0sq, scale, pad1, pad2;
};

constexpr unsigned kFlagSkip = 1u;   // no pixel of the tile is gated in (or bad navigation)
constexpr unsigned kFlagFull = 2u;   // every pixel of the tile is gated in
constexpr unsigned kFlagPoly = 4u;   // receiver offset by the series (degree 5, or 4 with kFlagDeg4)
constexpr unsigned kFlagDeg4 = 8u;   // the degree-4 series already meets the bound
constexpr int kEmptyRow = 30000;     // encodes an empty gate interval (never matches a local x)
constexpr double kPolyTol = 1e-8;    // metres, bound on the series truncation error
constexpr double kTrackTol = 2e-6;   // metres, bound on the departure of a position table from
                                     // the straight line a record uses for it

__device__ __forceinline__ double tile_centre(const SwathDev& sw, int a, int first, int extent) {
  return sw.o[a] + ((double)first + 0.5 * (double)(extent - 1)) * sw.d[a];
}

__device__ __forceinline__ bool finite3(double a, double b, double c) {
  return isfinite(a) && isfinite(b) && isfinite(c);
}

// Beam-gate class of the tile box for one cone apex X (Sec. II-C, with the
// transmitter and the receiver tested separately as in Sec. III-B). The cone
// |x - X_x| <= tan(g) rho, rho the (y, z) distance to X; over an axis-aligned
// box |x - X_x| and rho vary independently, so
//   out: min |dx| > tan(g) max rho,   in: max |dx| <= tan(g) min rho.
// Margins keep "in" and "out" strictly away from the cone surface; anything
// closer is "partial" and decided per row.
enum { kGateOut = 0, kGateIn = 1, kGatePartial = 2 };

__host__ __device__ inline int gate_class(double tan2, double x, double y, double z, double bx0, double bx1,
                                          double by0, double by1, double bz0, double bz1) {
  // squared form: out iff dxmin^2 > tan^2 rmax^2, in iff dxmax^2 <= tan^2 rmin^2
  const double dxmin = fmax(0.0, fmax(bx0 - x, x - bx1));
  const double dxmax = fmax(fabs(bx0 - x), fabs(bx1 - x));
  const double dymin = fmax(0.0, fmax(by0 - y, y - by1));
  const double dymax = fmax(fabs(by0 - y), fabs(by1 - y));
  const double dzmin = fmax(0.0, fmax(bz0 - z, z - bz1));
  const double dzmax = fmax(fabs(bz0 - z), fabs(bz1 - z));
  const double r2min = dymin * dymin + dzmin * dzmin;
  const double r2max = dymax * dymax + dzmax * dzmax;
  if (dxmin * dxmin > tan2 * r2max * (1.0 + 1e-11) + 1e-18) return kGateOut;
  if (dxmax * dxmax <= tan2 * r2min * (1.0 - 1e-11) - 1e-18) return kGateIn;
  return kGatePartial;
}

// Coarser per-(tile, ping) form used by the cull pass, with the box given by
// its pixel-centre extent [xa, xb] x [ya, yb] x [za, zb]: can any point of the
// box lie inside the cone of apex X? Uses the smallest |dx| and the largest
// rho over the box (each bounds its own coordinate, so the test is
// conservative: it may keep a box whose points all lie outside, never the
// reverse).
__host__ __device__ inline bool cone_may_hit(double tan_g, double xa, double xb, double ya, double yb, double za,
                                             double zb, const double* X) {
  const double dxm = fmax(0.0, fmax(xa - X[0], X[0] - xb));
  const double dy = fmax(fabs(ya - X[1]), fabs(yb - X[1]));
  const double dz = fmax(fabs(za - X[2]), fabs(zb - X[2]));
  const double rho = sqrt(dy * dy + dz * dz);
  return dxm <= tan_g * rho * (1.0 + 1e-9) + 1e-9;
}

// Position table (motion 2): ping p's displacement Delta(t) is linear between
// samples j h and (j + 1) h. The straight line through segment j, written
// Delta(t) = q + v t, and the segment that holds a delay tau (the first and
// last segments continue past the table's ends).
__device__ __forceinline__ void track_line(const SwathDev& sw, int p, int j, double q[3], double v[3]) {
  const double* a = sw.track + ((size_t)p * sw.track_n + j) * 3;
  const double t = (double)j * sw.track_h;
  for (int k = 0; k < 3; ++k) {
    v[k] = (a[3 + k] - a[k]) / sw.track_h;
    q[k] = a[k] - v[k] * t;
  }
}

__device__ __forceinline__ int track_segment_of(const SwathDev& sw, double tau) {
  const double u = floor(tau / sw.track_h);
  if (!(u >= 0.0)) return 0;                       // also a delay that is not finite
  return u >= (double)(sw.track_n - 2) ? sw.track_n - 2 : (int)u;
}

// The segment whose line ping p's records of the tile use: the one holding
// the tile centre's delay with the transmitter's own position standing for
// the receivers (they lie within the array's length of it), by fixed-point
// iteration on c tau = d_T + |C - T - Delta(tau)| (contraction |v| / c).
__device__ __forceinline__ int track_segment(const SwathDev& sw, int p, const double C[3], double c) {
  const double* T = sw.tx + (size_t)p * 3;
  const double u0 = C[0] - T[0], u1 = C[1] - T[1], u2 = C[2] - T[2];
  const double d = sqrt(u0 * u0 + u1 * u1 + u2 * u2);
  double tau = 2.0 * d / c;
  for (int it = 0; it < 12; ++it) {
    const int j = track_segment_of(sw, tau);
    double q[3], v[3];
    track_line(sw, p, j, q, v);
    const double w0 = u0 - q[0] - v[0] * tau, w1 = u1 - q[1] - v[1] * tau, w2 = u2 - q[2] - v[2] * tau;
    tau = (d + sqrt(w0 * w0 + w1 * w1 + w2 * w2)) / c;
  }
  return track_segment_of(sw, tau);
}

// Largest departure of ping p's table from the line of segment j over delays
// [ta, tb]: past each knot where the slope changes (t_{j+1} .. t_{N-2} above
// the segment, t_j .. t_1 below it) the table turns by at most A, the
// largest velocity change between neighbouring segments, so at distance d
// past the first such knot it is off by at most A sum_k (d - k h) over the
// knots passed.
__device__ __forceinline__ double track_line_error(const SwathDev& sw, int p, int j, double ta, double tb) {
  const double h = sw.track_h;
  const double A = (double)sw.tstats[p].y * (1.0 + 1e-6);
  double e = 0.0;
  const double db = tb - (double)(j + 1) * h;
  if (db > 0.0) {
    const double k = fmin(floor(db / h) + 1.0, (double)(sw.track_n - 2 - j));
    if (k > 0.0) e += A * (k * db - 0.5 * h * k * (k - 1.0));
  }
  const double da = (double)j * h - ta;
  if (da > 0.0) {
    const double k = fmin(floor(da / h) + 1.0, (double)j);
    if (k > 0.0) e += A * (k * da - 0.5 * h * k * (k - 1.0));
  }
  return e;
}

// Receiver record and window start for (ping p, element e) of the tile centred
// at C. Returns false if the navigation is not finite (record marked skip).
//
// MOTION (receivers moving during reception along the straight line
// R(t) = R + q + v t: a constant velocity v_p with q = 0, or segment jseg of
// the ping's position table): the reference delay is the exact root of
// c tau = d_T + |C - R - q - v tau| at the tile centre (the larger root of
// (c^2 - |v|^2) tau^2 - 2 (c d_T - a.v) tau + d_T^2 - |a|^2 = 0, a = C - R - q),
// *dc_out the extra path c tau - d_T - d_R it implies, and the window starts
// one sample earlier (the plan adds two samples to W). A bound on how much
// that extra path changes across the tile, r (2 W / (d_R - r) + 4 |v| / c)
// with W = |q| + |v| tau_max the line's largest displacement, must stay
// within one sample; for a table, the table's departure from the line over
// the tile's delays must stay within kTrackTol; otherwise, or for a line not
// finite or of |v| >= c / 2, the record is refused like bad navigation.
template <bool MOTION = false>
__device__ __forceinline__ bool make_rx_record(const SwathDev& sw, double inv_c, const double C[3], int p, int e,
                                               RxRec* rec, int* n0_out, double c = 0.0, float* dc_out = nullptr,
                                               int jseg = 0) {
  const double* T = sw.tx + (size_t)p * 3;
  const double* R = sw.rx + ((size_t)p * sw.E + e) * 3;
  const double tx0 = T[0], tx1 = T[1], tx2 = T[2];
  const double rx0 = R[0], rx1 = R[1], rx2 = R[2];
  const double uT0 = C[0] - tx0, uT1 = C[1] - tx1, uT2 = C[2] - tx2;
  const double uR0 = C[0] - rx0, uR1 = C[1] - rx1, uR2 = C[2] - rx2;
  const double d0T = sqrt(uT0 * uT0 + uT1 * uT1 + uT2 * uT2);
  const double d0R = sqrt(uR0 * uR0 + uR1 * uR1 + uR2 * uR2);
  bool ok = finite3(tx0, tx1, tx2) && finite3(rx0, rx1, rx2);
  double tau = (d0T + d0R) * inv_c;
  if constexpr (MOTION) {
    double q[3] = {0.0, 0.0, 0.0}, v[3];
    if (sw.motion == 2) {
      track_line(sw, p, jseg, q, v);
    } else {
      const double* V = sw.vel + (size_t)p * 3;
      v[0] = V[0];
      v[1] = V[1];
      v[2] = V[2];
    }
    const double v0 = v[0], v1 = v[1], v2 = v[2];
    const double a0 = uR0 - q[0], a1 = uR1 - q[1], a2 = uR2 - q[2];
    const double vv = v0 * v0 + v1 * v1 + v2 * v2;
    const double av = a0 * v0 + a1 * v1 + a2 * v2;
    const double A = c * c - vv;
    const double Bh = c * d0T - av;
    const double tm = (Bh + sqrt(Bh * Bh - A * (d0T * d0T - (a0 * a0 + a1 * a1 + a2 * a2)))) / A;
    const double r = sw.half_diag, vm = sqrt(vv);
    const double wm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]) + vm * (tm + 2.0 * r * inv_c);
    const double bound = r * (2.0 * wm / fmax(d0R - r, 1e-3) + 4.0 * vm * inv_c);
    ok = ok && finite3(v0, v1, v2) && finite3(q[0], q[1], q[2]) && vv < 0.25 * c * c && isfinite(tm) &&
         bound * sw.fs * inv_c <= 1.0;
    if (sw.motion == 2 && ok) {
      // the pixels' delays lie within 2 r / c of the centre's, plus the one
      // sample the motion path may change across the tile
      const double s = 2.0 * r * inv_c + 2.0 / sw.fs;
      ok = sw.tstats[p].w == 0.0f && track_line_error(sw, p, jseg, tm - s, tm + s) <= kTrackTol;
    }
    double dcm = 0.0;
    if (ok) {
      dcm = c * tm - d0T - d0R;
      tau = tm;
    }
    *dc_out = (float)dcm;
  }
  const double uref = (tau - sw.t0) * sw.fs;
  const double span = 2.0 * sw.half_diag * sw.fs * inv_c;
  double nstart = floor(uref - span) - (MOTION ? 3.0 : 2.0);
  if (!(nstart > -1.0e9)) nstart = -1.0e9;          // also maps NaN to a harmless value
  if (nstart > 1.0e9) nstart = 1.0e9;
  // window start even: staging loads two samples per lane, aligned
  int n0 = (int)nstart;
  n0 -= n0 & 1;
  const double cyc = sw.fc * tau;
  unsigned flags = ok ? 0u : kFlagSkip;
  // series bound over the tile: |num| <= 2 d0 r + r^2, remainder of
  // sqrt(1+y) - 1 after y^5 at most (21/1024) |y|^6 / (1 - |y|), after y^4 at
  // most (7/256) |y|^5 / (1 - |y|) (binomial coefficients of decreasing size)
  const double r = sw.half_diag;
  const double i1 = 1.0 / d0R, i2 = i1 * i1;
  const double y = (2.0 * d0R * r + r * r) * i2;
  double a1 = 0.0, a2 = 0.0, a3 = 0.0, a4 = 0.0, a5 = 0.0;
  const double y3 = y * y * y;
  if (ok && y < 0.5 && d0R * (21.0 / 1024.0) * (y3 * y3) <= kPolyTol * (1.0 - y)) {
    flags |= kFlagPoly;
    if (d0R * (7.0 / 256.0) * (y3 * y * y) <= kPolyTol * (1.0 - y)) flags |= kFlagDeg4;
    a1 = 0.5 * i1;
    a2 = -0.125 * i1 * i2;
    a3 = 0.0625 * i1 * i2 * i2;
    a4 = -(5.0 / 128.0) * i1 * i2 * i2 * i2;
    a5 = (7.0 / 256.0) * i1 * i2 * i2 * i2 * i2;
  }
  rec->q0 = make_float4((float)(2.0 * uR0), (float)(2.0 * uR1), (float)(2.0 * uR2), __uint_as_float(flags));
  rec->q1 = make_float4((float)(uref - (double)n0 - 0.5), (float)(cyc - floor(cyc)), (float)a5, (float)d0R);
  rec->q2 = make_float4((float)a1, (float)a2, (float)a3, (float)a4);
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
  rec->scale = sw.dtype == 0 ? 1.0f : sw.scale[p];
  rec->pad1 = rec->pad2 = 0.0f;
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

// Window entry and weight of a sample position with FP32 adds and one
// shift-add: adding 2^23 rounds sh = s - 1/2 to an integer n held in the low
// mantissa bits of t = sh + 2^23, and w = sh - n. The LDS byte address of entry
// n of a window at base is base + 16 n = (base - 16 bits(2^23)) + 16 bits(t)
// in 32-bit arithmetic, so window_base() folds the constant once per window.
// The window length is sized so that every pixel of the tile reads an entry in
// 0..W (W is the zero entry that gated-out pixels read).
constexpr float kRoundMagic = 8388608.0f;
constexpr unsigned kRoundMagicBits = 0x4B000000u;

__device__ __forceinline__ unsigned lds_address(const void* p) {
  return (unsigned)(uintptr_t)((__attribute__((address_space(3))) const void*)p);
}

__device__ __forceinline__ unsigned window_base(const float4* win) {
  return lds_address(win) - (kRoundMagicBits << 4);
}

__device__ __forceinline__ float4 window_read(unsigned wbase, float sh, float* w) {
  const float t = sh + kRoundMagic;
  *w = sh - (t - kRoundMagic);
  const unsigned addr = wbase + (__float_as_uint(t) << 4);
  typedef float f32x4 __attribute__((ext_vector_type(4)));
  const f32x4 q = *reinterpret_cast<__attribute__((address_space(3))) const f32x4*>((uintptr_t)addr);
  return make_float4(q.x, q.y, q.z, q.w);
}

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

// LDS layout for a chunk of NR (ping, element) records spanning at most NS
// pings, with window length W:
//   TxRec tx[NS]   RxRec rx[NR]   int n0[NR]   int rows[NR][ROWS] (gate only)
//   float4 win[NR][W+1]: {(E[n] + E[n+1]) / 2, E[n+1] - E[n]} for n < W,
//   entry W all zero.
// Interpolation at sample position s is then one 16-byte read and two FMAs:
// with n = round(s - 1/2) and w = (s - 1/2) - n in [-1/2, 1/2],
//   (1 - frac s) E[floor s] + frac(s) E[floor s + 1] = mid[n] + w diff[n]
// (a tie, s an integer rounded down to n = s - 1, gives w = 1/2 and the same
// value). Gated-out pixels read the zero entry.
struct LdsLayout {
  int off_tx, off_rx, off_n0, off_rows, off_win, off_dc, off_vel, bytes;
};

// Continuous motion appends the records' motion offsets (float [NR]) and the
// pings' receiver lines (3 float4 each [NS], as in the geometry region) after
// the windows.
__host__ __device__ inline LdsLayout lds_layout(int NR, int NS, int W, int ROWS, bool gate, bool motion = false) {
  LdsLayout L;
  int o = 0;
  L.off_tx = o;   o += NS * (int)sizeof(TxRec);
  L.off_rx = o;   o += NR * (int)sizeof(RxRec);
  L.off_n0 = o;   o += NR * 4;
  o = (o + 15) & ~15;
  L.off_rows = o; o += gate ? NR * ROWS * 4 : 0;
  o = (o + 15) & ~15;
  L.off_win = o;  o += NR * (W + 1) * 16;
  L.off_dc = o;   o += motion ? ((NR * 4 + 15) & ~15) : 0;
  L.off_vel = o;  o += motion ? NS * kMotionLineBytes : 0;
  L.bytes = o;
  return L;
}

static_assert(sizeof(RxRec) == kRxRecBytes, "receiver record size");
static_assert(sizeof(TxRec) == kTxRecBytes, "transmitter record size");

// This workgroup's geometry region (see geo_layout).
struct Geo {
  RxRec* rec;
  int* n0;
  TxRec* tx;
  int* rows;
  float* dc;      // continuous motion only
  float4* vel;    // 3 per ping: the receivers' line
};

__device__ __forceinline__ Geo geo_for(const Workspace& ws, const SwathDev& sw, int ROWS, bool gate) {
  const GeoLayout gl = geo_layout(sw.SC, sw.E, ROWS, gate, sw.motion != 0);
  unsigned char* base = ws.geo + (size_t)blockIdx.x * (size_t)ws.geo_stride;
  Geo g;
  g.rec = reinterpret_cast<RxRec*>(base + gl.rec);
  g.n0 = reinterpret_cast<int*>(base + gl.n0);
  g.tx = reinterpret_cast<TxRec*>(base + gl.tx);
  g.rows = reinterpret_cast<int*>(base + gl.rows);
  g.dc = reinterpret_cast<float*>(base + gl.dc);
  g.vel = reinterpret_cast<float4*>(base + gl.vel);
  return g;
}

// FP64 geometry of pings [P0, P0 + sc) of the tile whose first pixel is
// (x0, y0, z0): receiver and transmitter records, window starts, gate classes
// and, for every partially gated (ping, element), the exact gate interval of
// each pixel row. Built by the whole workgroup into its geometry region, so
// that the long FP64 dependency chains of many records overlap; the list of
// partial records is kept in LDS scratch (lpart, *lnpart) that the caller
// lends (the window area, unused between chunks). Ends with a barrier.
template <int NT, int TX, int LY, int LZ, bool GATE, bool MOTION = false>
__device__ __forceinline__ void build_geometry(const Geo& g, int* lpart, int* lnpart, const Workspace& ws,
                                               const SwathDev& sw, double c, const double* C, int P0, int sc,
                                               int x0, int y0, int z0, int tid) {
  constexpr int ROWS = LY * LZ;
  const int E = sw.E;
  const bool gate_on = GATE && sw.tan_g > 0.0;
  const double tan2 = sw.tan_g * sw.tan_g;
  const double inv_c = 1.0 / c;
  // pixel-centre box of the tile
  const double bx0 = sw.o[0] + (double)x0 * sw.d[0], bx1 = bx0 + (double)(TX - 1) * sw.d[0];
  const double by0 = sw.o[1] + (double)y0 * sw.d[1], by1 = by0 + (double)(LY - 1) * sw.d[1];
  const double bz0 = sw.o[2] + (double)z0 * sw.d[2], bz1 = bz0 + (double)(LZ - 1) * sw.d[2];
  if (tid == 0) *lnpart = 0;
  if (MOTION) {
    // each ping's receiver line first: the records of the ping share it
#pragma unroll 1
    for (int s = tid; s < sc; s += NT) {
      const int p = P0 + s;
      double q[3] = {0.0, 0.0, 0.0}, v[3];
      int j = 0;
      if (sw.motion == 2) {
        j = track_segment(sw, p, C, c);
        track_line(sw, p, j, q, v);
      } else {
        const double* V = sw.vel + (size_t)p * 3;
        v[0] = V[0];
        v[1] = V[1];
        v[2] = V[2];
      }
      g.vel[3 * s] = make_float4((float)v[0], (float)v[1], (float)v[2], (float)(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]));
      g.vel[3 * s + 1] = make_float4((float)q[0], (float)q[1], (float)q[2], (float)(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]));
      g.vel[3 * s + 2] = make_float4((float)(q[0] * v[0] + q[1] * v[1] + q[2] * v[2]), __int_as_float(j), 0.0f, 0.0f);
    }
  }
  __syncthreads();
#pragma unroll 1
  for (int r = tid; r < sc * E; r += NT) {
    const int slot = r / E, e = r - slot * E;
    const int p = P0 + slot;
    RxRec rec;
    int n0;
    float dcv = 0.0f;
    const int jseg = MOTION ? __float_as_int(g.vel[3 * slot + 2].y) : 0;
    if (!make_rx_record<MOTION>(sw, inv_c, C, p, e, &rec, &n0, c, &dcv, jseg)) atomicOr(&ws.counters[1], kStatusNav);
    if (MOTION) g.dc[r] = dcv;
    unsigned f = __float_as_uint(rec.q0.w);
    if (!gate_on) {
      f |= kFlagFull;
    } else if (sw.no_cull) {
      // no block classification: every record is decided row by row
      if (!(f & kFlagSkip)) lpart[atomicAdd(lnpart, 1)] = r;
    } else {
      const double* T = sw.tx + (size_t)p * 3;
      const double* R = sw.rx + ((size_t)p * E + e) * 3;
      const int gt = gate_class(tan2, T[0], T[1], T[2], bx0, bx1, by0, by1, bz0, bz1);
      const int gr = gt == kGateOut ? kGateOut : gate_class(tan2, R[0], R[1], R[2], bx0, bx1, by0, by1, bz0, bz1);
      if (gt == kGateOut || gr == kGateOut) f |= kFlagSkip;
      else if (gt == kGateIn && gr == kGateIn) f |= kFlagFull;
      if (!(f & (kFlagSkip | kFlagFull))) lpart[atomicAdd(lnpart, 1)] = r;
    }
    rec.q0.w = __uint_as_float(f);
    g.rec[r] = rec;
    g.n0[r] = n0;
  }
#pragma unroll 1
  for (int s = tid; s < sc; s += NT) make_tx_record(sw, C, P0 + s, &g.tx[s]);
  __syncthreads();
  if (gate_on) {
    const int np = *lnpart;
#pragma unroll 1
    for (int q = tid; q < np * ROWS; q += NT) {
      const int r = lpart[q / ROWS], rr = q % ROWS;
      const int slot = r / E, e = r - slot * E;
      const int ry = rr % LY, rz = rr / LY;
      const double y = sw.o[1] + (double)(y0 + ry) * sw.d[1];
      const double z = sw.o[2] + (double)(z0 + rz) * sw.d[2];
      g.rows[r * ROWS + rr] = gate_row(sw, P0 + slot, e, y, z, x0, TX);
    }
  }
  __syncthreads();
}


// Two consecutive complex samples from one load (16 bytes of FP32, or 8 bytes
// of 16-bit values dequantised with the ping's scale).
template <int DT>
struct PairLoad {
  typedef uint4 type;
};
template <>
struct PairLoad<1> {
  typedef uint2 type;
};
template <>
struct PairLoad<2> {
  typedef uint2 type;
};

__device__ __forceinline__ void unpack_pair(const uint4 q, float, float2* s) {
  s[0] = make_float2(__uint_as_float(q.x), __uint_as_float(q.y));
  s[1] = make_float2(__uint_as_float(q.z), __uint_as_float(q.w));
}

template <int DT>
__device__ __forceinline__ void unpack_pair16(const uint2 q, float scale, float2* s) {
  const unsigned w[2] = {q.x, q.y};
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    if (DT == 1) {
      typedef _Float16 h2 __attribute__((ext_vector_type(2)));
      const h2 v = __builtin_bit_cast(h2, w[i]);
      s[i] = make_float2((float)v.x * scale, (float)v.y * scale);
    } else {
      s[i] = make_float2(__uint_as_float(w[i] << 16) * scale, __uint_as_float(w[i] & 0xffff0000u) * scale);
    }
  }
}

__device__ __forceinline__ float2 load_guarded(const SwathDev& sw, size_t rowbase, int n, int dt, float scale) {
  if (n < 0 || n >= sw.Ns) return make_float2(0.0f, 0.0f);
  return load_sample(sw.echo, rowbase + (size_t)n, dt, scale);
}

// Ping slot x / E of chunk record x by a multiply with the FP32 reciprocal of
// E instead of an integer division (a long dependent sequence on the staging
// path): (x + 1/2) / E lies at least 1/(2E) from an integer, and the rounding
// of 1/E and of the product moves it by less than (x + 1/2) 2^-23 / E, so the
// truncation is exact for x < 2^21.
__device__ __forceinline__ int slot_of(int x, float invE) { return (int)(((float)x + 0.5f) * invE); }

// Echo windows of a chunk of nrows records into LDS; record r of the chunk is
// echo row row0 + r of the swath (rows in (ping, element) order), element e0
// + r of the chunk's first ping when r < E - e0, and its ping's transmitter
// record is ltx[(e0 + r) / E]. Entry k of window r holds the midpoint and the
// difference of E[n0+k] and E[n0+k+1] (k < W); entry W is zero.
// Each wave takes B windows (rows r = (ping, element) of the chunk) at a
// time and, per part of JS = 128 samples, issues the loads of all B rows
// before consuming any: a lane loads two consecutive samples and the sample
// after them (loaded, not taken from the next lane: a cross-lane shuffle
// would add an LDS round trip to the staging path). Row
// bookkeeping is wave-uniform and stays in scalar registers. Samples outside
// the record read as zero.
template <int NT, int DT, int SR = 3>
__device__ __forceinline__ void stage_windows(float4* lwin, const RxRec* lrx, const int* ln0, const TxRec* ltx,
                                              const SwathDev& sw, long long row0, int e0, int nrows, int tid,
                                              int lane, int wave_id) {
  typedef typename PairLoad<DT>::type LoadT;
  constexpr int NW = NT / 64;
  constexpr int SPL = 2;                    // samples per lane per load
  constexpr int JS = 64 * SPL;              // samples per part
  // rows in flight per wave: SR, so that a chunk spreads over the four waves
  // in even passes (24 records of the 2D tiles with three, 32 of the 3D
  // tiles with four; with eight, one wave of four sat idle on 24 records and
  // the staging spilled more registers)
  constexpr int B = SR;
  constexpr int SB = DT == 0 ? 8 : 4;       // bytes per sample
  const int wave = __builtin_amdgcn_readfirstlane(wave_id);
  const int E = sw.E, W = sw.W, Ns = sw.Ns;
  const float invE = 1.0f / (float)E;
  const int J = (W + JS) / JS;              // parts per window (samples 0..W)
  const bool aligned = (Ns % SPL) == 0;
  const char* echo = reinterpret_cast<const char*>(sw.echo);
  const int lane_off = SPL * lane;
#pragma unroll 1
  for (int r0 = wave * B; r0 < nrows; r0 += NW * B) {
#pragma unroll 1
    for (int part = 0; part < J; ++part) {
      LoadT q[B];
      float2 nxt[B];                        // the sample after the lane's pair (loaded, not shuffled)
      int first[B];                         // sample index of the part's first lane (uniform)
      float scl[B];                         // the row's ping scale (16-bit storage), read with the loads
      unsigned live = 0u, fast = 0u;        // per-row bits (uniform)
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int r = r0 + b;
        nxt[b] = make_float2(0.0f, 0.0f);
        first[b] = 0;
        scl[b] = 1.0f;
        if (r >= nrows) continue;
        const unsigned f = __builtin_amdgcn_readfirstlane(__float_as_uint(lrx[r].q0.w));
        if (f & kFlagSkip) continue;
        live |= 1u << b;
        first[b] = __builtin_amdgcn_readfirstlane(ln0[r]) + part * JS;
        if (DT != 0) scl[b] = ltx[slot_of(e0 + r, invE)].scale;
        if (aligned && first[b] >= 0 && first[b] + JS < Ns) {
          fast |= 1u << b;
          const size_t row = (size_t)(row0 + r) * (size_t)Ns + (size_t)first[b];
          q[b] = *reinterpret_cast<const LoadT*>(echo + (row + lane_off) * SB);
          nxt[b] = load_sample(sw.echo, row + lane_off + SPL, DT, 1.0f);
        }
      }
#pragma unroll
      for (int b = 0; b < B; ++b) {
        if (!(live & (1u << b))) continue;
        const int r = r0 + b;
        const size_t rowbase = (size_t)(row0 + r) * (size_t)Ns;
        const float scale = scl[b];
        const int n = first[b] + lane_off;
        float2 s[SPL + 1];
        if (fast & (1u << b)) {
          if constexpr (DT == 0) unpack_pair(q[b], scale, s);
          else unpack_pair16<DT>(q[b], scale, s);
        } else {
#pragma unroll
          for (int i = 0; i < SPL; ++i) s[i] = load_guarded(sw, rowbase, n + i, DT, scale);
        }
        s[SPL] = (fast & (1u << b)) ? make_float2(nxt[b].x * scale, nxt[b].y * scale)
                                    : load_guarded(sw, rowbase, n + SPL, DT, scale);
        float4* dst = lwin + (size_t)r * (W + 1) + part * JS;
#pragma unroll
        for (int i = 0; i < SPL; ++i) {
          if (part * JS + lane_off + i < W) {
            const float dr = s[i + 1].x - s[i].x, di = s[i + 1].y - s[i].y;
            dst[lane_off + i] = make_float4(fmaf(0.5f, dr, s[i].x), fmaf(0.5f, di, s[i].y), dr, di);
          }
        }
      }
    }
  }
  for (int r = tid; r < nrows; r += NT) lwin[(size_t)r * (W + 1) + W] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// Raw echo windows for the windowed-sinc variant: entry k of window r is the
// complex sample n0 - kSincHalf + k (zero outside the record), k = 0 ..
// W + 2 kSincHalf - 1, as float2 in the area that holds W + 1 float4 entries
// of the midpoint windows (W >= 7, so it has room). Row bookkeeping as in
// stage_windows; a lane loads and stores two consecutive samples.
template <int NT, int DT>
__device__ __forceinline__ void stage_windows_raw(float2* lwin, const RxRec* lrx, const int* ln0, const TxRec* ltx,
                                                  const SwathDev& sw, long long row0, int e0, int nrows, int lane,
                                                  int wave_id) {
  typedef typename PairLoad<DT>::type LoadT;
  constexpr int NW = NT / 64;
  constexpr int SPL = 2;
  constexpr int JS = 64 * SPL;
  // rows in flight per wave: six, one even pass over four waves for the
  // variant's 24-record chunks (81.5 ms against 84.3 ms with eight)
  constexpr int B = 6;
  constexpr int SB = DT == 0 ? 8 : 4;
  const int wave = __builtin_amdgcn_readfirstlane(wave_id);
  const int E = sw.E, Ns = sw.Ns;
  const float invE = 1.0f / (float)E;
  const int WR = sw.W + 2 * kSincHalf;     // entries per raw window
  const int stride = 2 * (sw.W + 1);       // float2 entries per record slot
  const int J = (WR + JS - 1) / JS;
  const bool aligned = (Ns % SPL) == 0;
  const char* echo = reinterpret_cast<const char*>(sw.echo);
  const int lane_off = SPL * lane;
#pragma unroll 1
  for (int r0 = wave * B; r0 < nrows; r0 += NW * B) {
#pragma unroll 1
    for (int part = 0; part < J; ++part) {
      LoadT q[B];
      int first[B];
      float scl[B];                         // the row's ping scale (16-bit storage), read with the loads
      unsigned live = 0u, fast = 0u;
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int r = r0 + b;
        first[b] = 0;
        scl[b] = 1.0f;
        if (r >= nrows) continue;
        const unsigned f = __builtin_amdgcn_readfirstlane(__float_as_uint(lrx[r].q0.w));
        if (f & kFlagSkip) continue;
        live |= 1u << b;
        first[b] = __builtin_amdgcn_readfirstlane(ln0[r]) - kSincHalf + part * JS;
        if (DT != 0) scl[b] = ltx[slot_of(e0 + r, invE)].scale;
        if (aligned && first[b] >= 0 && first[b] + JS <= Ns) {
          fast |= 1u << b;
          const size_t row = (size_t)(row0 + r) * (size_t)Ns + (size_t)first[b];
          q[b] = *reinterpret_cast<const LoadT*>(echo + (row + lane_off) * SB);
        }
      }
#pragma unroll
      for (int b = 0; b < B; ++b) {
        if (!(live & (1u << b))) continue;
        const int r = r0 + b;
        const size_t rowbase = (size_t)(row0 + r) * (size_t)Ns;
        const float scale = scl[b];
        const int n = first[b] + lane_off;
        float2 sm[SPL];
        if (fast & (1u << b)) {
          if constexpr (DT == 0) unpack_pair(q[b], scale, sm);
          else unpack_pair16<DT>(q[b], scale, sm);
        } else {
#pragma unroll
          for (int i = 0; i < SPL; ++i) sm[i] = load_guarded(sw, rowbase, n + i, DT, scale);
        }
        float2* dst = lwin + (size_t)r * stride + part * JS;
#pragma unroll
        for (int i = 0; i < SPL; ++i)
          if (part * JS + lane_off + i < WR) dst[lane_off + i] = sm[i];
      }
    }
  }
}

// The records of one chunk of a run whose geometry is in g: the nr records
// q0 .. q0 + nr - 1 of the run (record q is ping P0 + q / E, element q % E),
// spanning the ns pings s0 .. s0 + ns - 1 of the run. Receiver records,
// window starts, transmitter records and gate rows go into LDS. No barrier.
template <int NT, int ROWS, bool GATE, bool MOTION = false>
__device__ __forceinline__ void load_records(unsigned char* lds, const Geo& g, const SwathDev& sw, int q0, int nr,
                                             int s0, int ns, const LdsLayout& L, int tid) {
  TxRec* ltx = reinterpret_cast<TxRec*>(lds + L.off_tx);
  RxRec* lrx = reinterpret_cast<RxRec*>(lds + L.off_rx);
  int* ln0 = reinterpret_cast<int*>(lds + L.off_n0);
  const RxRec* grec = g.rec + q0;
  const int* gn0 = g.n0 + q0;
  for (int r = tid; r < nr; r += NT) {
    lrx[r] = grec[r];
    ln0[r] = gn0[r];
  }
  for (int s = tid; s < ns; s += NT) ltx[s] = g.tx[s0 + s];
  if (MOTION) {
    float* ldc = reinterpret_cast<float*>(lds + L.off_dc);
    float4* lvel = reinterpret_cast<float4*>(lds + L.off_vel);
    for (int r = tid; r < nr; r += NT) ldc[r] = g.dc[q0 + r];
    for (int s = tid; s < 3 * ns; s += NT) lvel[s] = g.vel[3 * s0 + s];
  }
  if (GATE && sw.tan_g > 0.0) {
    // rows of records that are not partial hold stale values and are never read
    const int4* src = reinterpret_cast<const int4*>(g.rows + (size_t)q0 * ROWS);
    int4* dst = reinterpret_cast<int4*>(lds + L.off_rows);
    for (int q = tid; q < nr * (ROWS / 4); q += NT) dst[q] = src[q];
  }
}

// One chunk (as for load_records): the records into LDS, then the echo
// windows (midpoint form, or raw samples for the windowed-sinc variant).
// Ends with a barrier.
template <int NT, int ROWS, bool GATE, int DT, bool RAW = false, bool MOTION = false, int SR = 3>
__device__ __forceinline__ void load_chunk(unsigned char* lds, const Geo& g, const SwathDev& sw, int P0, int q0,
                                           int nr, int s0, int ns, const LdsLayout& L, int tid, int lane,
                                           int wave) {
  load_records<NT, ROWS, GATE, MOTION>(lds, g, sw, q0, nr, s0, ns, L, tid);
  __syncthreads();
  if (RAW)
    stage_windows_raw<NT, DT>(reinterpret_cast<float2*>(lds + L.off_win), reinterpret_cast<const RxRec*>(lds + L.off_rx),
                              reinterpret_cast<const int*>(lds + L.off_n0), reinterpret_cast<const TxRec*>(lds + L.off_tx),
                              sw, (long long)P0 * sw.E + q0, q0 - s0 * sw.E, nr, lane, wave);
  else
    stage_windows<NT, DT, SR>(reinterpret_cast<float4*>(lds + L.off_win), reinterpret_cast<const RxRec*>(lds + L.off_rx),
                          reinterpret_cast<const int*>(lds + L.off_n0), reinterpret_cast<const TxRec*>(lds + L.off_tx),
                          sw, (long long)P0 * sw.E + q0, q0 - s0 * sw.E, nr, tid, lane, wave);
  __syncthreads();
}


}  // namespace sasbp

// Backprojection with sediment-water interface refraction in the propagation
// time (Sec. III-B: near-field sub-bottom imaging).
//
// The flat seafloor z = z_int separates water (sound speed c, above; the array
// is in the water) from sediment (c_sed, below). A leg from apex X to a pixel p
// below the interface crosses it at the point of least travel time, in the
// vertical plane through X and p at horizontal distance r from X, where
//     f(r) = r / (c a) - (D - r) / (c_sed b) = 0,   a = |(r, h1)|, b = |(D - r, h2)|
// (Snell's law; D the horizontal distance of X and p, h1 = z_int - X_z,
// h2 = p_z - z_int). The travel time t(r) = a / c + b / c_sed is convex with
// t' = f, so f grows with r and the root is its minimum. Legs to pixels at or
// above the interface are straight.
//
// Offset form. A workgroup's tile is a column of voxel levels; for each ping,
// element and level the workgroup first solves the leg to the tile's centre
// column at that level in FP64 (the reference: crossing r_c, legs a_c and b_c,
// time t_c, and the crossing's first and second derivatives in D by implicit
// differentiation of f(r(D), D) = 0), and keeps it in LDS. A pixel's leg then
// differs from the reference only through D (same h1, h2), and every quantity
// is carried as an FP32 offset that keeps its relative accuracy:
//     D^2 - D_c^2 = 2 (x_c - X_x) o_x + 2 (y_c - X_y) o_y + o_x^2 + o_y^2,
//     D - D_c = (D^2 - D_c^2) / (D + D_c),
//     a - a_c = (r - r_c)(r + r_c) / (a + a_c),   b - b_c = (u - u_c)(u + u_c) / (b + b_c),
// (o the pixel's offset from the column, u = D - r), so that the pixel's time
// is t_c + (a - a_c) / c + (b - b_c) / c_sed with t_c in FP64 and the offset
// in FP32. The crossing starts from the second-order expansion of r(D) about
// D_c; the start stands when it passes a certified bound: by convexity,
//     t(r) - t(r*) <= f(r)^2 / m,
// m a lower bound of f' between r and the root; the water leg's curvature
// h1^2 / (c a^3) over |r| <= D_c + rho (rho the tile's horizontal radius) is
// one. A start that passes keeps the time error below tt = 1e-5 of the
// shorter of the carrier and sampling periods. Otherwise (pixels near a sharp
// bend of r(D), just below the interface at the critical distance) the leg
// takes bracketed FP32 Newton steps (refine_crossing); a leg still
// unconverged after the step cap sets the plan's SAS_BP_ECONVERGE status. For
// faster sediment the bracket's upper end is the critical crossing.
//
// The sample position and the carrier phase are split the same way: each
// reference holds the whole samples and the fractions (of a sample, of a
// carrier cycle) of its leg's time, the pixel adds its FP32 offsets. The
// interpolation is linear in FP32 from the echo in global memory (L2-resident
// per tile). The beam gate keeps straight lines, tested in FP32 squares.
//
// Same persistent scheduling as the image kernel: a workgroup takes tiles from
// the cost-ordered list; lane (lx, ly, lz) owns K pixels of its row (a wave
// holds one level, so the references it reads are wave-uniform), loops over
// the tile's culled pings and every element, and writes each pixel once.
#include "tdbp_geom.h"

namespace sasbp {

constexpr int kRefractNewton = 24;     // most Newton steps of a leg that leaves its start
constexpr int kRefractRefs = 260;      // references per chunk: (elements + 1) x levels of a tile

// One leg's reference, to the tile's centre column at one voxel level (80 B).
struct RefractRef {
  float tdx, tdy;    // 2 (x_c - X_x), 2 (y_c - X_y)
  float d2c, dc;     // squared distance and distance to the centre: horizontal
                     // for a refracted leg, in 3D for a straight one
  float rc, rd, rdd; // crossing at the centre (an FP32 value), dr/dD, (d2r/dD2) / 2
  float h1s, h2s;    // h1^2, h2^2
  float ac, uc, bc;  // water leg, sediment run D_c - r_c and sediment leg at the centre
  float thr;         // certificate: tt m
  float hic;         // critical-crossing bound h1 c / sqrt(c_sed^2 - c^2) (infinite for slower sediment)
  float hsum;        // h1 + h2 (scale of the FP32 crossing resolution)
  float gz;          // dz^2 of a refracted leg (the gate's straight line), 0 for a straight one
  float fr, cy;      // fractions of the time in samples and in carrier cycles
  int n;             // whole samples
  int straight;      // 1: straight leg
};
static_assert(sizeof(RefractRef) == 80, "reference record size");

// Reciprocal square root in FP64 from the FP32 one and a Newton step
// y (3 - A y^2) / 2: relative error about 1.5 times the square of the FP32 one.
__device__ __forceinline__ double rsq_fp64(double A) {
  const double y = (double)__builtin_amdgcn_rsqf((float)A);
  return y * fma(-0.5 * A, y * y, 1.5);
}

// FP64 crossing at horizontal distance D: Newton steps kept inside the bracket
// [0, min(D, h1 rc_ratio)] (a step that leaves it is replaced by bisection)
// until a step is below FP64 resolution, from r = q D (q a nearby leg's
// crossing ratio; the straight-line crossing when q is outside [0, 1]). The
// step divides by f' in FP32 (a relative error of the step near 1e-7 still
// gains seven digits a step).
__device__ double crossing_fp64(double D, double h1, double h2, double inv_c, double inv_cs, double rc_ratio,
                                float q) {
  double lo = 0.0, hi = fmin(D, h1 * rc_ratio);
  const double q0 = (q >= 0.0f && q <= 1.0f) ? (double)q : h1 / (h1 + h2);
  double r = fmin(D * q0, hi);
  const double tol = 1e-14 * (D + h1 + h2), h1s = h1 * h1, h2s = h2 * h2;
  for (int it = 0; it < 80; ++it) {
    const double u = D - r;
    const double ia = rsq_fp64(fma(r, r, h1s)), ib = rsq_fp64(fma(u, u, h2s));
    const double f = r * ia * inv_c - u * ib * inv_cs;
    if (f < 0.0) lo = r; else hi = r;
    const double fp = h1s * ia * ia * ia * inv_c + h2s * ib * ib * ib * inv_cs;
    double rn = r - f * (double)__builtin_amdgcn_rcpf((float)fp);
    if (!(rn >= lo && rn <= hi)) rn = 0.5 * (lo + hi);
    const bool stop = !(fabs(rn - r) > tol);
    r = rn;
    if (stop) break;
  }
  return r;
}

// The reference of the leg from apex X to (xc, yc, pz), with its time split
// into whole samples and fractions (t_shift is subtracted from the time before
// the sample split: t0 for the transmit leg, 0 for a receiver leg). A
// non-finite apex sets bad and leaves an inert straight reference.
__device__ void refract_reference(RefractRef& R, double Xx, double Xy, double Xz, double xc, double yc, double pz,
                                  double rho, const SwathDev& sw, double inv_c, double inv_cs, double rc_ratio,
                                  double tt, double t_shift, float q_start, bool& bad) {
  RefractRef q;
  q.rc = q.rd = q.rdd = q.h1s = q.h2s = q.ac = q.uc = q.bc = q.thr = q.hic = q.hsum = q.gz = 0.0f;
  if (!finite3(Xx, Xy, Xz)) {
    bad = true;
    q.tdx = q.tdy = q.d2c = q.dc = q.fr = q.cy = 0.0f;
    q.n = -(1 << 29);   // every tap outside the row
    q.straight = 1;
    R = q;
    return;
  }
  const double dx = xc - Xx, dy = yc - Xy, dz = pz - Xz;
  const double h1 = sw.z_int - Xz, h2 = pz - sw.z_int;
  q.tdx = (float)(2.0 * dx);
  q.tdy = (float)(2.0 * dy);
  double t;
  if (!(h1 > 0.0) || !(h2 > 0.0)) {
    const double R2 = dx * dx + dy * dy + dz * dz, Rr = sqrt(R2);
    q.d2c = (float)R2;
    q.dc = (float)Rr;
    q.straight = 1;
    t = Rr * inv_c;
  } else {
    const double D = sqrt(dx * dx + dy * dy);
    const float rcf = (float)crossing_fp64(D, h1, h2, inv_c, inv_cs, rc_ratio, q_start);
    const double r = rcf, u = D - r;
    const double a = sqrt(r * r + h1 * h1), b = sqrt(u * u + h2 * h2);
    t = a * inv_c + b * inv_cs;
    // r(D) from f(r(D), D) = 0: with P = h1^2 / (c a^3), Q = h2^2 / (c_sed b^3),
    // f_r = P + Q, f_D = -Q, r' = Q / (P + Q); differentiating again,
    // r'' = -(P_r r'^2 + Q1 (1 - r')^2) / (P + Q), P_r = -3 h1^2 r / (c a^5),
    // Q1 = 3 h2^2 u / (c_sed b^5)
    const double a2 = a * a, b2 = b * b;
    const double P = h1 * h1 / (a2 * a) * inv_c, Q = h2 * h2 / (b2 * b) * inv_cs, Fr = P + Q;
    const double rd = Q / Fr;
    const double Pr = -3.0 * h1 * h1 * r / (a2 * a2 * a) * inv_c, Q1 = 3.0 * h2 * h2 * u / (b2 * b2 * b) * inv_cs;
    const double rdd = -(Pr * rd * rd + Q1 * (1.0 - rd) * (1.0 - rd)) / Fr;
    const double Dm = D + rho, am2 = Dm * Dm + h1 * h1;
    q.d2c = (float)(D * D);
    q.dc = (float)D;
    q.rc = rcf;
    q.rd = (float)rd;
    q.rdd = (float)(0.5 * rdd);
    q.h1s = fmaxf((float)(h1 * h1), 1e-30f);
    q.h2s = fmaxf((float)(h2 * h2), 1e-30f);
    q.ac = (float)a;
    q.uc = (float)u;
    q.bc = (float)b;
    q.thr = (float)(tt * h1 * h1 / (am2 * sqrt(am2)) * inv_c);   // tt x least water-leg curvature
    q.hic = (float)(h1 * rc_ratio);
    q.hsum = (float)(h1 + h2);
    q.gz = (float)(dz * dz);
    q.straight = 0;
  }
  const double s = (t - t_shift) * sw.fs, sn = floor(s);
  q.n = (int)fmin(fmax(sn, -5e8), 5e8);
  q.fr = (float)(s - sn);
  const double cyc = sw.fc * t;
  q.cy = (float)(cyc - floor(cyc));
  R = q;
}

// Bracketed FP32 Newton steps for a leg whose start failed the certificate.
// Stop tests: the certified bound f^2 <= tt m, m the water leg's curvature at
// r when the root lies below r (f > 0), at r = D otherwise; or a Newton step s
// that is small against the sediment leg b at the point it left (s <= b / 4,
// so that the local model holds over the step) and either bounds the time
// error f' s^2 / 2 below tt or reaches the FP32 resolution of r. The root lies
// in [0, D] and, for faster sediment, below the critical crossing hic (there
// f >= 0); without that bound a pixel just below the interface beyond the
// critical distance stalls near r = D, where the sediment leg is shorter than
// the step.
__device__ __forceinline__ float refine_crossing(float r, float D, float h1s, float h2s, float hic, float hsum,
                                                 float icf, float icsf, float tt, bool& conv) {
  const float iaD = __builtin_amdgcn_rsqf(fmaf(D, D, h1s));
  const float mD = h1s * iaD * iaD * iaD * icf;   // water-leg curvature at r = D (its smallest)
  float lo = 0.0f, hi = fminf(D, hic * (1.0f + 1e-6f));
  r = fminf(fmaxf(r, 0.0f), hi);   // a NaN start goes to 0
  const float tol = 1e-6f * (D + hsum);
  bool done = false;
  for (int it = 0; it < kRefractNewton; ++it) {
    const float u = D - r;
    const float ia = __builtin_amdgcn_rsqf(fmaf(r, r, h1s));
    const float ib = __builtin_amdgcn_rsqf(fmaf(u, u, h2s));
    const float f = r * ia * icf - u * ib * icsf;
    const float fw = h1s * ia * ia * ia * icf;
    const bool cert = f * f <= tt * (f >= 0.0f ? fw : mD);
    lo = f < 0.0f ? r : lo;
    hi = f < 0.0f ? hi : r;
    const float fp = fw + h2s * ib * ib * ib * icsf;
    float rn = r - f * __builtin_amdgcn_rcpf(fp);
    rn = ((rn >= lo) & (rn <= hi)) ? rn : 0.5f * (lo + hi);
    const float st = fabsf(rn - r);
    done = cert | ((st * ib <= 0.25f) & ((st <= tol) | (0.5f * fp * st * st <= tt)));
    r = cert ? r : rn;
    if (done) break;
  }
  conv = conv && done;
  return fminf(fmaxf(r, 0.0f), D);
}

// Travel-time offsets (s) of a lane's K pixels on one leg against the leg's
// reference, with D^2 (or the 3D squared distance of a straight leg) for the
// gate. (ox[k], oy): the pixels' horizontal offsets from the centre column,
// oo[k] = ox[k]^2 + oy^2.
template <int K>
__device__ __forceinline__ void leg_offsets(const RefractRef& R, const float (&ox)[K], float oy, const float (&oo)[K],
                                            float icf, float icsf, float tt, bool& conv, float (&dt)[K],
                                            float (&d2)[K]) {
  const float tdx = R.tdx, dc = R.dc, d2c = R.d2c;
  const float ty = R.tdy * oy;
  float dD[K], D[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const float num = fmaf(tdx, ox[k], ty + oo[k]);
    d2[k] = d2c + num;
    D[k] = d2[k] * __builtin_amdgcn_rsqf(fmaxf(d2[k], 1e-30f));
    dD[k] = num * __builtin_amdgcn_rcpf(dc + D[k]);
  }
  if (R.straight) {
#pragma unroll
    for (int k = 0; k < K; ++k) dt[k] = dD[k] * icf;
    return;
  }
  const float rc = R.rc, rd = R.rd, rdd = R.rdd, h1s = R.h1s, h2s = R.h2s, ac = R.ac, uc = R.uc, bc = R.bc;
  const float thr = R.thr;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    float r = __builtin_amdgcn_fmed3f(fmaf(dD[k], fmaf(rdd, dD[k], rd), rc), 0.0f, D[k]);   // warm start in [0, D]
    float u = D[k] - r;
    float A = fmaf(r, r, h1s), B = fmaf(u, u, h2s);
    float ia = __builtin_amdgcn_rsqf(A), ib = __builtin_amdgcn_rsqf(B);
    const float f = fmaf(r * ia, icf, -(u * ib) * icsf);
    if (!(f * f <= thr)) {
      r = refine_crossing(r, D[k], h1s, h2s, R.hic, R.hsum, icf, icsf, tt, conv);
      u = D[k] - r;
      A = fmaf(r, r, h1s);
      B = fmaf(u, u, h2s);
      ia = __builtin_amdgcn_rsqf(A);
      ib = __builtin_amdgcn_rsqf(B);
    }
    const float dr = r - rc, du = dD[k] - dr;
    const float sa = fmaf(A, ia, ac), sb = fmaf(B, ib, bc);   // a + a_c, b + b_c
    const float q = __builtin_amdgcn_rcpf(sa * sb);
    const float da = dr * (r + rc) * sb, db = du * (u + uc) * sa;
    dt[k] = fmaf(da, icf, db * icsf) * q;
  }
}

template <int L, bool GATE, int DT>
// Five waves per SIMD (96 VGPRs; a few values spill outside the inner loop):
// 0.81 s against 0.84 s at the four that 117 VGPRs allowed on the 3D volume.
__global__ __launch_bounds__(kLayouts[L].LX * kLayouts[L].LY * kLayouts[L].LZ)
__attribute__((amdgpu_waves_per_eu(5, 5))) void refract_kernel(
    Workspace ws, const SwathDev* __restrict__ swaths, const int* __restrict__ order,
    const int* __restrict__ tile_swath, const PingRange* __restrict__ prange, int n_tiles) {
  constexpr int K = kLayouts[L].K, LX = kLayouts[L].LX, LY = kLayouts[L].LY;
  constexpr int TX = LX * K, TY = LY, TZ = kLayouts[L].LZ, NT = LX * LY * TZ;
  constexpr int CE = kRefractRefs / TZ - 1;   // elements per chunk
  static_assert((LX * LY) % 64 == 0, "a wave holds one voxel level");
  static_assert(TX % 2 == 0 && TY % 2 == 0, "no pixel on the centre column");
  __shared__ RefractRef s_ref[kRefractRefs];
  __shared__ int s_item, s_bad;
  const int tid = threadIdx.x;
  const int lx = tid % LX, ly = (tid / LX) % LY, lz = tid / (LX * LY);
  for (;;) {
    __syncthreads();
    if (tid == 0) {
      s_item = next_tile(ws, blockIdx.x % kXcds);
      s_bad = 0;
    }
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);
    if (item < 0) break;
    const int t = __builtin_amdgcn_readfirstlane(order[item]);
    const int s = __builtin_amdgcn_readfirstlane(tile_swath[t]);
    const SwathDev& sw = swaths[s];
    const int lt = t - sw.tile0;
    const int tix = lt % sw.ntx, tiy = (lt / sw.ntx) % sw.nty, tiz = lt / (sw.ntx * sw.nty);
    const int iy = tiy * TY + ly, iz = tiz * TZ + lz;
    const double c = *sw.c;
    const double inv_c = 1.0 / c, inv_cs = 1.0 / sw.c_sed;
    const double ttd = 1e-5 / (sw.fc > sw.fs ? sw.fc : sw.fs);   // time error bound of a leg (s)
    const float tt = (float)ttd;
    const double rc_ratio = sw.c_sed > c ? c / sqrt(sw.c_sed * sw.c_sed - c * c) : __builtin_inf();
    const float icf = (float)inv_c, icsf = (float)inv_cs, fsf = (float)sw.fs, fcf = (float)sw.fc;
    const float s2 = (float)(sw.sin_g * sw.sin_g);
    const bool gate = GATE && sw.tan_g > 0.0;
    const int E = sw.E, Ns = sw.Ns;
    const void* const echo = sw.echo;
    bool conv = true;
    const PingRange pr = prange[t];
    // the centre column and the lane's offsets from it (exact in FP64, rounded once)
    const double xc = tile_centre(sw, 0, tix * TX, TX), yc = tile_centre(sw, 1, tiy * TY, TY);
    const double rho = (1.0 + 1e-6) * sqrt(0.25 * ((TX - 1) * sw.d[0]) * ((TX - 1) * sw.d[0]) +
                                           0.25 * ((TY - 1) * sw.d[1]) * ((TY - 1) * sw.d[1]));
    const float oy = (float)(sw.o[1] + (double)iy * sw.d[1] - yc);
    float ox[K], oo[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      ox[k] = (float)(sw.o[0] + (double)(tix * TX + lx + LX * k) * sw.d[0] - xc);
      oo[k] = fmaf(ox[k], ox[k], oy * oy);
    }
    float accr[K], acci[K], sT[K], cT[K];
    bool gT[K];
#pragma unroll
    for (int k = 0; k < K; ++k) { accr[k] = 0.0f; acci[k] = 0.0f; sT[k] = 0.0f; cT[k] = 0.0f; gT[k] = true; }
    int nT = 0;
    for (int p = pr.lo; p <= pr.hi; ++p) {
      const float scale = DT == 0 ? 1.0f : sw.scale[p];
      for (int e0 = 0; e0 < E; e0 += CE) {
        const int ce = min(CE, E - e0);
        __syncthreads();   // the previous chunk's references are consumed
        bool bad = false;
        for (int j = tid; j < (ce + 1) * TZ; j += NT) {
          const int leg = j / TZ, lev = j % TZ;
          if (leg == 0 && e0 != 0) continue;   // the transmit leg once per ping
          const double pz = sw.o[2] + (double)(tiz * TZ + lev) * sw.d[2];
          const double* X = leg == 0 ? sw.tx + (size_t)p * 3 : sw.rx + ((size_t)p * E + e0 + leg - 1) * 3;
          // the slot's previous leg (the same element and level one ping
          // back when a ping fits one chunk) starts the crossing
          const RefractRef& prev = s_ref[j];
          const float q0 = prev.straight == 0 && prev.dc > 0.0f ? prev.rc / prev.dc : -1.0f;
          refract_reference(s_ref[j], X[0], X[1], X[2], xc, yc, pz, rho, sw, inv_c, inv_cs, rc_ratio, ttd,
                            leg == 0 ? sw.t0 : 0.0, q0, bad);
        }
        if (bad) s_bad = 1;
        __syncthreads();
        if (e0 == 0) {
          float dtT[K], d2[K];
          const RefractRef& R = s_ref[lz];
          leg_offsets<K>(R, ox, oy, oo, icf, icsf, tt, conv, dtT, d2);
          const float fr = R.fr, cy = R.cy, hx = 0.5f * R.tdx, gz = R.gz;
          nT = R.n;
#pragma unroll
          for (int k = 0; k < K; ++k) {
            sT[k] = fmaf(dtT[k], fsf, fr);
            cT[k] = fmaf(dtT[k], fcf, cy);
            const float h = hx + ox[k];
            gT[k] = !gate || h * h <= s2 * (d2[k] + gz);
          }
        }
        for (int j = 0; j < ce; ++j) {
          const RefractRef& R = s_ref[(1 + j) * TZ + lz];
          float dt[K], d2[K];
          leg_offsets<K>(R, ox, oy, oo, icf, icsf, tt, conv, dt, d2);
          const float fr = R.fr, cy = R.cy, hx = 0.5f * R.tdx, gz = R.gz;
          const int n0 = nT + R.n;
          const size_t row = ((size_t)p * E + e0 + j) * (size_t)Ns;
#pragma unroll
          for (int k = 0; k < K; ++k) {
            bool g = gT[k];
            if (gate) {
              const float h = hx + ox[k];
              g = g && h * h <= s2 * (d2[k] + gz);
            }
            if (!g) continue;
            const float sp = fmaf(dt[k], fsf, sT[k]) + fr;   // sample position past n0
            const float fl = floorf(sp);
            const float w = sp - fl;
            const int n = n0 + (int)fl;
            float2 a = make_float2(0.0f, 0.0f), b = make_float2(0.0f, 0.0f);
            if ((unsigned)n < (unsigned)Ns) a = load_sample(echo, row + (size_t)n, DT, scale);
            if ((unsigned)(n + 1) < (unsigned)Ns) b = load_sample(echo, row + (size_t)(n + 1), DT, scale);
            const float vr = fmaf(w, b.x - a.x, a.x), vi = fmaf(w, b.y - a.y, a.y);
            const float cyc = __builtin_amdgcn_fractf(fmaf(dt[k], fcf, cT[k]) + cy);
            const float sn = __builtin_amdgcn_sinf(cyc), cs = __builtin_amdgcn_cosf(cyc);
            accr[k] = fmaf(vr, cs, fmaf(-vi, sn, accr[k]));
            acci[k] = fmaf(vr, sn, fmaf(vi, cs, acci[k]));
          }
        }
      }
    }
    __syncthreads();   // every reference write (and s_bad) seen
    const bool bad = s_bad != 0;
    if (bad && tid == 0) atomicOr(&ws.counters[1], kStatusNav);
    if (!conv) atomicOr(&ws.counters[1], kStatusConverge);
    if (iy < sw.ny && iz < sw.nz) {
      float2* out = sw.image + ((size_t)iz * sw.ny + iy) * (size_t)sw.nx;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int ix = tix * TX + lx + LX * k;
        if (ix < sw.nx) out[ix] = bad ? make_float2(0.0f, 0.0f) : make_float2(accr[k], acci[k]);
      }
    }
  }
}

typedef void (*RefractKernelFn)(Workspace, const SwathDev*, const int*, const int*, const PingRange*, int);

template <int L>
static RefractKernelFn refract_for_layout(bool gate, int dt) {
  if (gate) return dt == 0 ? refract_kernel<L, true, 0> : dt == 1 ? refract_kernel<L, true, 1> : refract_kernel<L, true, 2>;
  return dt == 0 ? refract_kernel<L, false, 0> : dt == 1 ? refract_kernel<L, false, 1> : refract_kernel<L, false, 2>;
}

RefractKernelFn refract_kernel_for(int layout, bool gate, int dt) {
  switch (layout) {
    case 0: return refract_for_layout<0>(gate, dt);
    case 1: return refract_for_layout<1>(gate, dt);
    case 2: return refract_for_layout<2>(gate, dt);
    case 3: return refract_for_layout<3>(gate, dt);
    case 4: return refract_for_layout<4>(gate, dt);
    case 5: return refract_for_layout<5>(gate, dt);
    case 6: return refract_for_layout<6>(gate, dt);
    case 7: return refract_for_layout<7>(gate, dt);
    case 8: return refract_for_layout<8>(gate, dt);
    default: return nullptr;
  }
}

}  // namespace sasbp

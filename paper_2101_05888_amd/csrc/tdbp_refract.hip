// Backprojection with sediment-water interface refraction in the propagation
// time (Sec. III-B: near-field sub-bottom imaging).
//
// The flat seafloor z = z_int separates water (sound speed c, above; the array
// is in the water) from sediment (c_sed, below). A leg from apex X to a pixel p
// below the interface crosses it at the point of least travel time, in the
// vertical plane through X and p at horizontal distance r from X, where
//     f(r) = r / (c a) - (D - r) / (c_sed b) = 0,   a = |(r, h1)|, b = |(D - r, h2)|
// (Snell's law; D the horizontal distance of X and p, h1 = z_int - X_z,
// h2 = p_z - z_int). f grows with r, so Newton steps kept inside the bracket
// [0, D] that the sign of f shrinks converge; the travel time a / c + b / c_sed
// is stationary at the root, so a few steps give it to FP32 rounding. A pixel's
// transmit leg starts from the straight-line crossing r = D h1 / (h1 + h2); its
// receiver legs start from the crossing ratio r / D of the leg before (the
// transmit leg, then the previous element), which neighbouring apexes nearly
// share. The loop stops once the travel-time error is below 1e-5 of the
// shorter of the carrier and sampling periods, by a certified bound from the
// convexity of the travel time or by the local model of a small Newton step
// (details at refracted_time): about 1.3 steps per leg on the near-interface
// scenes, up to about fifteen for pixels just below the interface at the
// critical distance. For faster sediment the bracket's upper end is the
// critical crossing. A leg still unconverged after the step cap sets the
// plan's SAS_BP_ECONVERGE status. Legs to
// pixels at or above the interface are straight. The beam gate keeps straight lines.
//
// Precision: the crossing point by FP32 Newton steps, the leg times (square
// roots from the FP32 reciprocal square root and one FP64 Newton step), the
// delay and the carrier phase (reduced to revolutions) in FP64; the interpolation is
// linear in FP32, the echo read from global memory (L2-resident per tile).
//
// Same persistent scheduling as the image kernel: a workgroup takes tiles from
// the cost-ordered list; lane (lx, ly, lz) owns K pixels of its row, loops over
// the tile's culled pings and every element, and writes each pixel once.
#include "tdbp_geom.h"

namespace sasbp {

constexpr int kRefractNewton = 24;  // most Newton steps per leg (most stop after one or two)

// Square root of A >= 0 in FP64 from the FP32 reciprocal square root y and one
// Newton step s + (A - s^2) y / 2 with s = A y: the relative error, about the
// square of the FP32 one, stays near 1e-13 (the seed is kept finite for an A
// below the FP32 range, so A = 0 gives 0).
__device__ __forceinline__ double sqrt_refined(double A) {
  const double y = (double)__builtin_amdgcn_rsqf(fmaxf((float)A, 1e-30f));
  const double s = A * y;
  return fma(fma(-s, s, A), 0.5 * y, s);
}

// One leg's travel time (FP64 result): the crossing distance r by FP32 Newton
// steps from the ratio q = r / D (in: a nearby leg's, out: this leg's) until
// the time error is below tt seconds, then the time at r evaluated in FP64
// (it is stationary in r, so the error of r reaches it only squared).
//
// Stop tests. The travel time t(r) is convex (t' = f, f' > 0), so at any r
//     t(r) - t(r*) <= |f(r)| |r - r*| <= f(r)^2 / m,
// m a lower bound of f' between r and the root r*; the water leg's curvature
// h1^2 / (c a^3) is one, smallest where a is largest: at r when the root lies
// below r (f > 0), at r = D otherwise. A leg stops when f^2 <= tt m there
// (certified), or when a Newton step s is small against the sediment leg b
// at the point it left (s <= b / 4, so that the local model holds over the
// step) and either bounds the time error f' s^2 / 2 below tt or reaches the
// FP32 resolution of r.
//
// The root lies in [0, D] and, when the sediment is faster (c_sed > c), also
// below the critical crossing r_c = h1 c / sqrt(c_sed^2 - c^2): there f >= 0
// (the water leg is at the critical angle, the sediment leg's sine is at most
// one). rc_ratio = c / sqrt(c_sed^2 - c^2) (infinite for slower sediment).
// Without that bound, a pixel just below the interface beyond the critical
// distance starts near r = D, where the sediment leg is shorter than the step
// and Newton steps stall at a point far from the root. A leg that meets no
// stop test within kRefractNewton steps clears *conv.
__device__ __forceinline__ double refracted_time(double dx, double dy, double dz, double h1, double h2, double inv_c,
                                                 double inv_cs, float rc_ratio, float tt, float& q, bool& conv) {
  const double D2 = dx * dx + dy * dy;
  if (!(h2 > 0.0) || !(h1 > 0.0))   // pixel at or above the interface (or apex below it): straight
    return sqrt_refined(D2 + dz * dz) * inv_c;
  const double D = sqrt_refined(D2);   // enters the leg time at first order: kept to FP64 accuracy
  const float Df = (float)D, h1f = (float)h1, h2f = (float)h2, icf = (float)inv_c, icsf = (float)inv_cs;
  const float h1s = h1f * h1f;
  const float iaD = __builtin_amdgcn_rsqf(fmaf(Df, Df, h1s));
  const float mD = h1s * iaD * iaD * iaD * icf;    // water-leg curvature at r = D (its smallest)
  float lo = 0.0f, hi = fminf(Df, h1f * rc_ratio * (1.0f + 1e-6f));
  float r = fminf(fmaxf(q * Df, 0.0f), hi);   // a NaN ratio starts at 0
  const float tol = 1e-6f * (Df + h1f + h2f);   // FP32 resolution of the crossing
  bool done = false;
  for (int it = 0; it < kRefractNewton; ++it) {
    const float u = Df - r;
    const float ia = __builtin_amdgcn_rsqf(fmaf(r, r, h1s));
    const float ib = __builtin_amdgcn_rsqf(fmaf(u, u, h2f * h2f));
    const float f = r * ia * icf - u * ib * icsf;
    const float fw = h1s * ia * ia * ia * icf;
    const bool cert = f * f <= tt * (f >= 0.0f ? fw : mD);   // certified: r stays
    lo = f < 0.0f ? r : lo;
    hi = f < 0.0f ? hi : r;
    const float fp = fw + h2f * h2f * ib * ib * ib * icsf;
    float rn = r - f * __builtin_amdgcn_rcpf(fp);
    rn = ((rn >= lo) & (rn <= hi)) ? rn : 0.5f * (lo + hi);   // a converged step may land on the bracket end
    const float st = fabsf(rn - r);
    // every test evaluated, combined without short-circuit branches
    done = cert | ((st * ib <= 0.25f) & ((st <= tol) | (0.5f * fp * st * st <= tt)));
    r = cert ? r : rn;
    if (done) break;
  }
  conv = conv && done;
  if (Df > 0.0f) q = r * __builtin_amdgcn_rcpf(Df);   // only the next leg's starting point
  const double rd = fmin((double)r, D), ud = D - rd;   // FP32 rounding may put r past D
  return sqrt_refined(rd * rd + h1 * h1) * inv_c + sqrt_refined(ud * ud + h2 * h2) * inv_cs;
}

template <int L, bool GATE, int DT>
__global__ __launch_bounds__(kLayouts[L].LX * kLayouts[L].LY * kLayouts[L].LZ) void refract_kernel(
    Workspace ws, const SwathDev* __restrict__ swaths, const int* __restrict__ order,
    const int* __restrict__ tile_swath, const PingRange* __restrict__ prange, int n_tiles) {
  constexpr int K = kLayouts[L].K, LX = kLayouts[L].LX, LY = kLayouts[L].LY;
  constexpr int TX = LX * K, TY = LY, TZ = kLayouts[L].LZ;
  const int tid = threadIdx.x;
  const int lx = tid % LX, ly = (tid / LX) % LY, lz = tid / (LX * LY);
  __shared__ int s_item;
  for (;;) {
    __syncthreads();
    if (tid == 0) s_item = next_tile(ws, blockIdx.x % kXcds);
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
    const float tt = (float)(1e-5 / (sw.fc > sw.fs ? sw.fc : sw.fs));   // time error bound of a stopped solve (s)
    const float rc_ratio = sw.c_sed > c ? (float)(c / sqrt(sw.c_sed * sw.c_sed - c * c)) : __builtin_inff();
    bool conv = true;
    const PingRange pr = prange[t];
    // pixel centres (FP64)
    double px[K];
    const double py = sw.o[1] + (double)iy * sw.d[1], pz = sw.o[2] + (double)iz * sw.d[2];
#pragma unroll
    for (int k = 0; k < K; ++k) px[k] = sw.o[0] + (double)(tix * TX + lx + LX * k) * sw.d[0];
    float accr[K], acci[K];
#pragma unroll
    for (int k = 0; k < K; ++k) { accr[k] = 0.0f; acci[k] = 0.0f; }
    bool bad = false;
    for (int p = pr.lo; p <= pr.hi; ++p) {
      const double* T = sw.tx + (size_t)p * 3;
      const double Tx = T[0], Ty = T[1], Tz = T[2];
      bad |= !(finite3(Tx, Ty, Tz));
      const float scale = sw.dtype == 0 ? 1.0f : sw.scale[p];
      double tT[K];
      bool gT[K];
      float q[K];   // crossing ratio of the pixel's last leg
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const double dx = px[k] - Tx, dy = py - Ty, dz = pz - Tz;
        const double h1 = sw.z_int - Tz, h2 = pz - sw.z_int;
        q[k] = (float)(h1 / (h1 + h2));   // straight-line crossing
        tT[k] = refracted_time(dx, dy, dz, h1, h2, inv_c, inv_cs, rc_ratio, tt, q[k], conv);
        gT[k] = true;
        if (GATE && sw.tan_g > 0.0) gT[k] = fabs(dx) <= sw.sin_g * sqrt(dx * dx + dy * dy + dz * dz);
      }
      for (int e = 0; e < sw.E; ++e) {
        const double* R = sw.rx + ((size_t)p * sw.E + e) * 3;
        const double Rx = R[0], Ry = R[1], Rz = R[2];
        bad |= !(finite3(Rx, Ry, Rz));
        const size_t row = ((size_t)p * sw.E + e) * (size_t)sw.Ns;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const double dx = px[k] - Rx, dy = py - Ry, dz = pz - Rz;
          bool g = gT[k];
          if (GATE && sw.tan_g > 0.0) g = g && fabs(dx) <= sw.sin_g * sqrt(dx * dx + dy * dy + dz * dz);
          if (!g) continue;
          const double tau = tT[k] + refracted_time(dx, dy, dz, sw.z_int - Rz, pz - sw.z_int, inv_c, inv_cs,
                                                    rc_ratio, tt, q[k], conv);
          const double u = (tau - sw.t0) * sw.fs;
          const double nf = floor(u);
          const float w = (float)(u - nf);
          const int n = (int)fmin(fmax(nf, -2.0), (double)sw.Ns);   // outside the row (or NaN): both taps zero
          float2 a = make_float2(0.0f, 0.0f), b = make_float2(0.0f, 0.0f);
          if (n >= 0 && n < sw.Ns) a = load_sample(sw.echo, row + (size_t)n, DT, scale);
          if (n + 1 >= 0 && n + 1 < sw.Ns) b = load_sample(sw.echo, row + (size_t)(n + 1), DT, scale);
          const float vr = fmaf(w, b.x - a.x, a.x), vi = fmaf(w, b.y - a.y, a.y);
          const double cyc_d = sw.fc * tau;
          const float cyc = (float)(cyc_d - floor(cyc_d));
          const float sn = __builtin_amdgcn_sinf(cyc), cs = __builtin_amdgcn_cosf(cyc);
          accr[k] = fmaf(vr, cs, fmaf(-vi, sn, accr[k]));
          acci[k] = fmaf(vr, sn, fmaf(vi, cs, acci[k]));
        }
      }
    }
    if (bad) atomicOr(&ws.counters[1], kStatusNav);
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

// Geometry adjoint (vector-Jacobian product), exact gated-term count and the
// image-sharpness objective used for data-driven motion estimation (the paper
// estimates sway and heave from the sonar data itself, Sec. I and II-D).
//
// For a cotangent Gbar (Gbar = dJ/dRe I + j dJ/dIm I) every term of the
// backprojection sum contributes coef = Re(conj(Gbar(p)) D) with
//     D = dI/dtau = [f_s (E[n+1] - E[n]) + j 2 pi f_c L] exp(j 2 pi f_c tau),
// and dtau/dR = (R - p)/(c d_R), dtau/dT = (T - p)/(c d_T), dtau/dc = -tau/c.
// The kernel replays the image kernel's traversal (same tiles, records, gate
// rows and LDS windows), recomputing delays instead of storing them. Per
// (tile, ping, element) it reduces over the tile's pixels
//     S0 = sum coef/d_R, S = sum coef/d_R * delta, C0 = sum coef, C1 = sum coef * Delta
// (delta = pixel offset from the tile centre, Delta = FP32 two-way path
// offset) and turns them into FP64 gradient partials with the tile's FP64
// reference geometry:
//     dJ/dR += -(u_R S0 + S) / c,   u_R = C - R,
//     dJ/dc += -(tau_ref C0 + C1 / c) / c.
// A second kernel sums the partials over tiles in tile order, so the result is
// bitwise reproducible.
#include "tdbp_geom.h"

namespace sasbp {

// One DPP-moved operand per step (no LDS round trip, unlike a shuffle):
// xor 1 and 2 within quads, the half-row and row mirrors give every lane its
// 16-lane row sum, then row broadcasts of lanes 15 and 31 fold the rows into
// lane 63, which is read out. A fixed order, so the sum is reproducible.
// Needs every lane of the wave active.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_move(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xf, false));
}
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_move<0xb1, 0xf>(v);    // quad_perm [1, 0, 3, 2]
  v += dpp_move<0x4e, 0xf>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp_move<0x141, 0xf>(v);   // row_half_mirror
  v += dpp_move<0x140, 0xf>(v);   // row_mirror
  v += dpp_move<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_move<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

// Extra LDS after the image layout: per (slot, element, wave) 6 floats of
// receiver/sound-speed sums and per (slot, wave) 4 floats of transmitter sums.
__host__ __device__ inline int adjoint_red_offset(int CP, int E, int W, int ROWS, bool gate) {
  return (lds_layout(CP * E, CP, W, ROWS, gate).bytes + 15) & ~15;
}
__host__ __device__ inline int adjoint_bytes(int CP, int E, int W, int ROWS, bool gate, int NW) {
  return adjoint_red_offset(CP, E, W, ROWS, gate) + CP * E * NW * 6 * 4 + CP * NW * 4 * 4;
}

template <int L, bool GATE, int DT>
__global__ __launch_bounds__(kLayouts[L].LX * kLayouts[L].LY * kLayouts[L].LZ)
__attribute__((amdgpu_waves_per_eu(kAdjointWaves, kAdjointWaves))) void adjoint_kernel(
    Workspace ws, const SwathDev* __restrict__ swaths, const int* __restrict__ order,
    const int* __restrict__ tile_swath, const PingRange* __restrict__ prange, int n_tiles) {
  extern __shared__ __align__(16) unsigned char lds[];
  constexpr int K = kLayouts[L].K, LX = kLayouts[L].LX, LY = kLayouts[L].LY, LZ = kLayouts[L].LZ;
  constexpr int NT = LX * LY * LZ, NW = NT / 64;
  constexpr int TX = LX * K, TY = LY, TZ = LZ, ROWS = LY * LZ;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lx = tid % LX, ly = (tid / LX) % LY, lz = tid / (LX * LY);
  const int row = ly + LY * lz;
  __shared__ int s_item;
  __shared__ int s_npart;

  for (;;) {
    __syncthreads();
    if (tid == 0) s_item = next_tile(ws, blockIdx.x % kXcds);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);
    if (item < 0) break;
    const int t = __builtin_amdgcn_readfirstlane(order[item]);
    const int s = __builtin_amdgcn_readfirstlane(tile_swath[t]);
    const SwathDev& sw = swaths[s];
    const int E = sw.E, W = sw.W, CP = sw.CP;
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
    const float fsf = (float)sw.fs;
    const float tpf = (float)(2.0 * 3.14159265358979323846 * sw.fc);
    const PingRange pr = prange[t];
    const LdsLayout Ld = lds_layout(CP * E, CP, W, ROWS, GATE);
    const TxRec* ltx = reinterpret_cast<const TxRec*>(lds + Ld.off_tx);
    const RxRec* lrx = reinterpret_cast<const RxRec*>(lds + Ld.off_rx);
    const int* lrows = reinterpret_cast<const int*>(lds + Ld.off_rows);
    const float4* lwin = reinterpret_cast<const float4*>(lds + Ld.off_win);
    float* red = reinterpret_cast<float*>(lds + adjoint_red_offset(CP, E, W, ROWS, GATE));
    float* redt = red + CP * E * NW * 6;

    const float sx = (float)sw.d[0], sy = (float)sw.d[1], sz = (float)sw.d[2];
    float dx[K], dsq[K], gr[K], gi[K];
    const float dyl = (float)(2 * ly - (TY - 1)) * 0.5f * sy;
    const float dzl = (float)(2 * lz - (TZ - 1)) * 0.5f * sz;
    const int iy = y0 + ly, iz = z0 + lz;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      dx[k] = (float)(2 * (lx + LX * k) - (TX - 1)) * 0.5f * sx;
      dsq[k] = dx[k] * dx[k] + dyl * dyl + dzl * dzl;
      const int ix = x0 + lx + LX * k;
      float2 g = make_float2(0.0f, 0.0f);
      if (ix < sw.nx && iy < sw.ny && iz < sw.nz) g = sw.gimage[((size_t)iz * sw.ny + iy) * (size_t)sw.nx + ix];
      gr[k] = g.x;
      gi[k] = g.y;
    }
    const float szero = (float)W;

    const Geo geo = geo_for(ws, sw, ROWS, GATE);
    int* lpart = reinterpret_cast<int*>(lds + Ld.off_win);   // window area, free between chunks

    for (int P0 = pr.lo; P0 <= pr.hi; P0 += sw.SC) {
     const int sc = min(sw.SC, pr.hi - P0 + 1);
     __syncthreads();
     build_geometry<NT, TX, LY, LZ, GATE>(geo, lpart, &s_npart, ws, sw, c, C, P0, sc, x0, y0, z0, tid);
     for (int off = 0; off < sc; off += CP) {
      const int cp = min(CP, sc - off);
      const int p0 = P0 + off;
      if (off > 0) __syncthreads();
      load_chunk<NT, ROWS, GATE, DT>(lds, geo, sw, P0, off * E, cp * E, off, cp, Ld, tid, lane, wave);
      for (int slot = 0; slot < cp; ++slot) {
        const TxRec tr = ltx[slot];
        const float tyz = fmaf(tr.uy2, dyl, tr.uz2 * dzl);
        float dT[K], qsum[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const float num = fmaf(tr.ux2, dx[k], tyz + dsq[k]);
          const float sq = __builtin_amdgcn_sqrtf(tr.d0sq + num);
          dT[k] = num * __builtin_amdgcn_rcpf(tr.d0 + sq);
          qsum[k] = 0.0f;
        }
        for (int e = 0; e < E; ++e) {
          const int r = slot * E + e;
          const RxRec rec = lrx[r];
          const unsigned f = __builtin_amdgcn_readfirstlane(__float_as_uint(rec.q0.w));
          float S0 = 0.0f, Sx = 0.0f, C0 = 0.0f, C1 = 0.0f;
          if (!(f & kFlagSkip)) {
            const bool test = GATE && !(f & kFlagFull);
            int da = 0, span = 0;
            if (test) {
              const int v = lrows[r * ROWS + row];
              const int a = row_lo(v), b = row_hi(v);
              da = lx - a;
              span = b - a;
            }
            const float ryz = fmaf(rec.q0.y, dyl, rec.q0.z * dzl);
            const float d0 = rec.q1.w;
            const float d0sq = d0 * d0;
            const float4* win = lwin + (size_t)r * (W + 1);
            // delays first, then every window read in flight at once, then
            // the per-pixel terms (as in the image kernel)
            float dRk[K], Dk[K], sidx[K], cyc[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
              const float num = fmaf(rec.q0.x, dx[k], ryz + dsq[k]);
              const float sq = __builtin_amdgcn_sqrtf(d0sq + num);
              dRk[k] = num * __builtin_amdgcn_rcpf(d0 + sq);
              Dk[k] = dT[k] + dRk[k];
              float si = fmaf(Dk[k], fs_c, rec.q1.x);
              cyc[k] = fmaf(Dk[k], fc_c, rec.q1.y);
              if (test) {
                const bool in = (unsigned)(da + LX * k) <= (unsigned)span;
                si = in ? si : szero;
              }
              sidx[k] = si;
            }
            float4 vk[K];
            float wk[K];
            const unsigned wbase = window_base(win);
#pragma unroll
            for (int k = 0; k < K; ++k) vk[k] = window_read(wbase, sidx[k], &wk[k]);
#pragma unroll
            for (int k = 0; k < K; ++k) {
              const float D = Dk[k], dR = dRk[k], wt = wk[k];
              const float4 v = vk[k];
              const float sn = __builtin_amdgcn_sinf(cyc[k]);
              const float cs = __builtin_amdgcn_cosf(cyc[k]);
              const float dar = v.z, dai = v.w;
              const float Lr = fmaf(wt, dar, v.x), Li = fmaf(wt, dai, v.y);
              const float Xr = fmaf(fsf, dar, -tpf * Li);
              const float Xi = fmaf(fsf, dai, tpf * Lr);
              const float Dr = fmaf(Xr, cs, -Xi * sn);
              const float Di = fmaf(Xr, sn, Xi * cs);
              const float coef = fmaf(gr[k], Dr, gi[k] * Di);
              const float q = coef * __builtin_amdgcn_rcpf(d0 + dR);
              S0 += q;
              Sx = fmaf(q, dx[k], Sx);
              C0 += coef;
              C1 = fmaf(coef, D, C1);
              qsum[k] += coef;
            }
          }
          if (!(f & kFlagSkip)) {
            const float Sy = S0 * dyl, Sz = S0 * dzl;
            const float v0 = wave_sum(S0), v1 = wave_sum(Sx), v2 = wave_sum(Sy), v3 = wave_sum(Sz);
            const float v4 = wave_sum(C0), v5 = wave_sum(C1);
            if (lane == 0) {
              float* o = red + ((size_t)r * NW + wave) * 6;
              o[0] = v0; o[1] = v1; o[2] = v2; o[3] = v3; o[4] = v4; o[5] = v5;
            }
          } else if (lane == 0) {
            float* o = red + ((size_t)r * NW + wave) * 6;
            o[0] = o[1] = o[2] = o[3] = o[4] = o[5] = 0.0f;
          }
        }
        // transmitter: coef summed over elements, weighted by 1/d_T per pixel
        float T0 = 0.0f, Tx = 0.0f;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const float q = qsum[k] * __builtin_amdgcn_rcpf(tr.d0 + dT[k]);
          T0 += q;
          Tx = fmaf(q, dx[k], Tx);
        }
        const float t0 = wave_sum(T0), t1 = wave_sum(Tx), t2 = wave_sum(T0 * dyl), t3 = wave_sum(T0 * dzl);
        if (lane == 0) {
          float* o = redt + ((size_t)slot * NW + wave) * 4;
          o[0] = t0; o[1] = t1; o[2] = t2; o[3] = t3;
        }
      }
      __syncthreads();
      // FP64 partials of this chunk: fixed order over the four waves
      for (int r = tid; r < cp * E; r += NT) {
        const int slot = r / E, e = r - slot * E;
        const int p = p0 + slot;
        double a[6] = {0, 0, 0, 0, 0, 0};
        for (int w = 0; w < NW; ++w)
          for (int j = 0; j < 6; ++j) a[j] += (double)red[((size_t)r * NW + w) * 6 + j];
        const double* T = sw.tx + (size_t)p * 3;
        const double* R = sw.rx + ((size_t)p * E + e) * 3;
        const double uR0 = C[0] - R[0], uR1 = C[1] - R[1], uR2 = C[2] - R[2];
        const double uT0 = C[0] - T[0], uT1 = C[1] - T[1], uT2 = C[2] - T[2];
        const double d0R = sqrt(uR0 * uR0 + uR1 * uR1 + uR2 * uR2);
        const double d0T = sqrt(uT0 * uT0 + uT1 * uT1 + uT2 * uT2);
        const double tau = (d0T + d0R) / c;
        double* out = ws.partials + ((size_t)sw.part_off + ((size_t)lt * sw.P + p) * E + e) * kPartial;
        out[0] = -(uR0 * a[0] + a[1]) / c;
        out[1] = -(uR1 * a[0] + a[2]) / c;
        out[2] = -(uR2 * a[0] + a[3]) / c;
        out[3] = -(tau * a[4] + a[5] / c) / c;
        if (e == 0) {
          double b[4] = {0, 0, 0, 0};
          for (int w = 0; w < NW; ++w)
            for (int j = 0; j < 4; ++j) b[j] += (double)redt[((size_t)slot * NW + w) * 4 + j];
          out[4] = -(uT0 * b[0] + b[1]) / c;
          out[5] = -(uT1 * b[0] + b[2]) / c;
          out[6] = -(uT2 * b[0] + b[3]) / c;
        } else {
          out[4] = out[5] = out[6] = 0.0;
        }
        out[7] = 0.0;
      }
     }
    }
  }
}

// Sum the partials over tiles (tile order) for each (swath, ping): thread e
// owns element e; element 0 also carries the transmitter sums. The
// sound-speed partials are summed over elements in order into cpart.
__global__ __launch_bounds__(kThreads) void adjoint_reduce_kernel(Workspace ws, int max_p) {
  const int s = blockIdx.y;
  const SwathDev& sw = ws.swaths[s];
  const int p = blockIdx.x;
  __shared__ double cred[kMaxElem];
  if (p >= sw.P) return;
  const int E = sw.E;
  const int nt = sw.ntx * sw.nty * sw.ntz;
  for (int e = threadIdx.x; e < E; e += blockDim.x) {
    double g[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int lt = 0; lt < nt; ++lt) {
      const PingRange pr = ws.prange[sw.tile0 + lt];
      if (p < pr.lo || p > pr.hi) continue;
      const double* in = ws.partials + ((size_t)sw.part_off + ((size_t)lt * sw.P + p) * E + e) * kPartial;
      for (int j = 0; j < 7; ++j) g[j] += in[j];
    }
    double* gr = sw.grad_rx + ((size_t)p * E + e) * 3;
    gr[0] = g[0];
    gr[1] = g[1];
    gr[2] = g[2];
    cred[e] = g[3];
    if (e == 0) {
      double* gt = sw.grad_tx + (size_t)p * 3;
      gt[0] = g[4];
      gt[1] = g[5];
      gt[2] = g[6];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double acc = 0.0;
    for (int e = 0; e < E; ++e) acc += cred[e];
    ws.cpart[(size_t)s * max_p + p] = acc;
  }
}

__global__ void adjoint_c_kernel(Workspace ws, int max_p) {
  const int s = blockIdx.x;
  const SwathDev& sw = ws.swaths[s];
  if (threadIdx.x == 0) {
    double acc = 0.0;
    for (int p = 0; p < sw.P; ++p) acc += ws.cpart[(size_t)s * max_p + p];
    sw.grad_c[0] = acc;
  }
}

// Exact count of gated-in terms of swath s: per (ping, element, image row) the
// x-interval of the cone intersection, clipped to the image.
__global__ __launch_bounds__(kThreads) void count_kernel(Workspace ws, int s, long long total,
                                                         unsigned long long* out) {
  const SwathDev& sw = ws.swaths[s];
  const int rows = sw.ny * sw.nz;
  unsigned long long acc = 0;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (long long)gridDim.x * blockDim.x) {
    const long long pe = q / rows;
    const int rr = (int)(q - pe * rows);
    const int p = (int)(pe / sw.E), e = (int)(pe - (long long)p * sw.E);
    const int iy = rr % sw.ny, iz = rr / sw.ny;
    const double y = sw.o[1] + (double)iy * sw.d[1];
    const double z = sw.o[2] + (double)iz * sw.d[2];
    const double* T = sw.tx + (size_t)p * 3;
    const double* R = sw.rx + ((size_t)p * sw.E + e) * 3;
    const double hT = sw.tan_g * sqrt((y - T[1]) * (y - T[1]) + (z - T[2]) * (z - T[2]));
    const double hR = sw.tan_g * sqrt((y - R[1]) * (y - R[1]) + (z - R[2]) * (z - R[2]));
    const double lo = fmax(T[0] - hT, R[0] - hR);
    const double hi = fmin(T[0] + hT, R[0] + hR);
    const double a = fmax(ceil((lo - sw.o[0]) / sw.d[0]), 0.0);
    const double b = fmin(floor((hi - sw.o[0]) / sw.d[0]), (double)(sw.nx - 1));
    if (a <= b) acc += (unsigned long long)(b - a + 1.0);
  }
  __shared__ unsigned long long part[kThreads];
  part[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long sum = 0;
    for (int i = 0; i < (int)blockDim.x; ++i) sum += part[i];
    atomicAdd(out, sum);
  }
}

__global__ void zero_u64(unsigned long long* p) { *p = 0ull; }

// Sharpness S = A / B^2 with A = sum |I|^4, B = sum |I|^2 (FP64, fixed order),
// and optionally the cotangent Gbar = 4 I (|I|^2 / B^2 - A / B^3).
// kSharpBlocks (tdbp_dev.h) partial pairs, then the two sums in a fixed order.

__global__ __launch_bounds__(kThreads) void sharp_partial_kernel(const float2* img, long long n, double* partials) {
  double a = 0.0, b = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float2 v = img[i];
    const double m = (double)v.x * v.x + (double)v.y * v.y;
    b += m;
    a += m * m;
  }
  __shared__ double sa[kThreads], sb[kThreads];
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sa[threadIdx.x] += sa[threadIdx.x + h];
      sb[threadIdx.x] += sb[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = sa[0];
    partials[2 * blockIdx.x + 1] = sb[0];
  }
}

__global__ void sharp_final_kernel(const double* partials, double* ab, double* out_S) {
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int i = 0; i < kSharpBlocks; ++i) {
      a += partials[2 * i];
      b += partials[2 * i + 1];
    }
    ab[0] = a;
    ab[1] = b;
    out_S[0] = b > 0.0 ? a / (b * b) : 0.0;
  }
}

__global__ __launch_bounds__(kThreads) void sharp_grad_kernel(const float2* img, long long n, const double* ab,
                                                              float2* grad) {
  const double A = ab[0], B = ab[1];
  const double inv_b2 = B > 0.0 ? 1.0 / (B * B) : 0.0;
  const double k2 = B > 0.0 ? A / (B * B * B) : 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float2 v = img[i];
    const double m = (double)v.x * v.x + (double)v.y * v.y;
    const double f = 4.0 * (m * inv_b2 - k2);
    grad[i] = make_float2((float)(f * v.x), (float)(f * v.y));
  }
}

// ------------------------------------------------------------ dispatch ---

typedef void (*AdjointKernelFn)(Workspace, const SwathDev*, const int*, const int*, const PingRange*, int);

template <int L>
static AdjointKernelFn adjoint_for_layout(bool gate, int dt) {
  if (gate) {
    switch (dt) {
      case 0: return adjoint_kernel<L, true, 0>;
      case 1: return adjoint_kernel<L, true, 1>;
      default: return adjoint_kernel<L, true, 2>;
    }
  }
  switch (dt) {
    case 0: return adjoint_kernel<L, false, 0>;
    case 1: return adjoint_kernel<L, false, 1>;
    default: return adjoint_kernel<L, false, 2>;
  }
}

AdjointKernelFn adjoint_kernel_for(int layout, bool gate, int dt) {
  switch (layout) {
    case 0: return adjoint_for_layout<0>(gate, dt);
    case 1: return adjoint_for_layout<1>(gate, dt);
    case 2: return adjoint_for_layout<2>(gate, dt);
    case 3: return adjoint_for_layout<3>(gate, dt);
    case 4: return adjoint_for_layout<4>(gate, dt);
    case 5: return adjoint_for_layout<5>(gate, dt);
    case 6: return adjoint_for_layout<6>(gate, dt);
    case 7: return adjoint_for_layout<7>(gate, dt);
    case 8: return adjoint_for_layout<8>(gate, dt);
    default: return nullptr;
  }
}

int adjoint_lds_bytes(int CP, int E, int W, int ROWS, bool gate, int threads) {
  return adjoint_bytes(CP, E, W, ROWS, gate, threads / 64);
}

hipError_t launch_adjoint(AdjointKernelFn fn, const Workspace& ws, int n_tiles, int grid, int threads, int lds_bytes,
                          hipStream_t st) {
  hipLaunchKernelGGL(fn, dim3(grid), dim3(threads), lds_bytes, st, ws, (const SwathDev*)ws.swaths,
                     (const int*)ws.order, (const int*)ws.tile_swath, (const PingRange*)ws.prange, n_tiles);
  return hipGetLastError();
}

hipError_t adjoint_occupancy(AdjointKernelFn fn, int threads, int lds_bytes, int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, threads, lds_bytes);
}

hipError_t set_adjoint_lds_limit(AdjointKernelFn fn, int lds_bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                             lds_bytes);
}

hipError_t launch_adjoint_reduce(const Workspace& ws, int n_swaths, int max_p, hipStream_t st) {
  hipLaunchKernelGGL(adjoint_reduce_kernel, dim3(max_p, n_swaths), dim3(kThreads), 0, st, ws, max_p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(adjoint_c_kernel, dim3(n_swaths), dim3(64), 0, st, ws, max_p);
  return hipGetLastError();
}

hipError_t launch_count(const Workspace& ws, int s, int P, int E, int rows, unsigned long long* out,
                        hipStream_t st) {
  hipLaunchKernelGGL(zero_u64, dim3(1), dim3(1), 0, st, out);
  const long long total = (long long)P * E * rows;
  long long blocks = (total + kThreads - 1) / kThreads;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(count_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, st, ws, s, total, out);
  return hipGetLastError();
}

hipError_t launch_sharpness(const void* image, long long n, double* partials, double* out_S, void* grad,
                            hipStream_t st) {
  const float2* img = reinterpret_cast<const float2*>(image);
  hipLaunchKernelGGL(sharp_partial_kernel, dim3(kSharpBlocks), dim3(kThreads), 0, st, img, n, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  double* ab = partials + 2 * kSharpBlocks;
  hipLaunchKernelGGL(sharp_final_kernel, dim3(1), dim3(64), 0, st, partials, ab, out_S);
  e = hipGetLastError();
  if (e != hipSuccess || !grad) return e;
  long long blocks = (n + kThreads - 1) / kThreads;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(sharp_grad_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, st, img, n, ab,
                     reinterpret_cast<float2*>(grad));
  return hipGetLastError();
}

}  // namespace sasbp

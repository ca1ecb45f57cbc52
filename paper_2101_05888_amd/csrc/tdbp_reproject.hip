// Reprojection: the linear adjoint of the image with respect to the echo.
//
// The image is complex-linear in the echo cube (Eq. 1 inverted, Sec. II-A):
// I = A E, where a term (pixel p, ping i, element e) with g = 1 reads
// (1 - w) E[n] + w E[n+1] at n = floor(u) and multiplies it by
// exp(+j 2 pi f_c tau). The adjoint A^H Y of an image-shaped Y scatters
//     (1 - w) exp(-j 2 pi f_c tau) Y(p)  to sample n,
//     w       exp(-j 2 pi f_c tau) Y(p)  to sample n + 1
// of row (i, e), dropping samples outside the record. For Y = Gbar
// (dJ/dRe I + j dJ/dIm I) this is the gradient of J with respect to the
// echo in the same convention.
//
// The kernel replays the image kernel's traversal (tiles in cost order,
// runs of FP64 geometry, chunks of (ping, element) records, the same FP32
// delay offsets and rounded sample position) but, instead of reading an echo
// window, each record owns an LDS accumulator window of complex samples. Each
// lane adds its K pixels' two weighted contributions with LDS integer
// atomics, in fixed point: a tile's contributions are scaled by
// s = 2^30 / (pixels x max |Re, Im Y| over the tile), so that no window sum
// can reach 2^31, and rounded to integers (a resolution of about 1e-6 of the
// tile's largest Y). Integer sums are exact and order-free; LDS float atomics
// measured over ten times slower here. After the chunk the windows are
// scaled back and added into the output cube with global float atomics, whose
// order across tiles depends on scheduling: results agree with the FP64
// definition to FP32 rounding but are not bitwise reproducible.
#include "tdbp_geom.h"

namespace sasbp {

// Accumulator entry k of a record's window is sample n0 + k, k = 0 .. W + 1
// (W + 2 complex values as int32 pairs), in the LDS area the image kernel
// uses for its W + 1 float4 echo entries.
typedef __attribute__((address_space(3))) int LdsInt;
typedef __attribute__((address_space(1))) float GlobalFloat;

__device__ __forceinline__ void lds_add(unsigned addr, float v) {
  __hip_atomic_fetch_add(reinterpret_cast<LdsInt*>((uintptr_t)addr), (int)rintf(v), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void global_add(float* p, float v) {
  __hip_atomic_fetch_add(reinterpret_cast<GlobalFloat*>(reinterpret_cast<uintptr_t>(p)), v, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
}

// One (ping, element) record applied to the K pixels of a lane: delay offsets
// exactly as the image kernel forms them, then the conjugate phasor times Y
// (already multiplied by the tile's fixed-point scale) split over the two
// samples around the sample position. Gated-out pixels add zero at the window
// end (entries W, W + 1).
template <int K, int LX, int DEG, bool TEST>
__device__ __forceinline__ void scatter(const RxRec& rec, unsigned acc_base, const float* dx, const float* dsq,
                                        const float* dT, float dyl, float dzl, float fs_c, float fc_c, float szero,
                                        int da, int span, const float* yr, const float* yi) {
  const float ryz = fmaf(rec.q0.y, dyl, rec.q0.z * dzl);
  const float d0 = rec.q1.w;
  const float d0sq = d0 * d0;
  float sidx[K], cyc[K], keep[K];
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
    float si = fmaf(D, fs_c, rec.q1.x);   // sample position - 1/2 in the window
    cyc[k] = fmaf(D, fc_c, rec.q1.y);
    keep[k] = 1.0f;
    if (TEST) {
      const bool in = (unsigned)(da + LX * k) <= (unsigned)span;
      si = in ? si : szero;
      keep[k] = in ? 1.0f : 0.0f;
    }
    sidx[k] = si;
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    // n = round(s - 1/2), wm = (s - 1/2) - n in [-1/2, 1/2]: weights 1/2 - wm
    // on sample n and 1/2 + wm on sample n + 1 (the image kernel's midpoint
    // form of (1 - w, w))
    const float t = sidx[k] + kRoundMagic;
    const float wm = sidx[k] - (t - kRoundMagic);
    const unsigned addr = acc_base + (__float_as_uint(t) << 3);
    const float sn = __builtin_amdgcn_sinf(cyc[k]);
    const float cs = __builtin_amdgcn_cosf(cyc[k]);
    const float xr = keep[k] * fmaf(cs, yr[k], sn * yi[k]);    // Re(exp(-j phi) Y)
    const float xi = keep[k] * fmaf(cs, yi[k], -sn * yr[k]);   // Im(exp(-j phi) Y)
    const float a = 0.5f - wm, b = 0.5f + wm;
    lds_add(addr, a * xr);
    lds_add(addr + 4, a * xi);
    lds_add(addr + 8, b * xr);
    lds_add(addr + 12, b * xi);
  }
}

template <int L, bool GATE>
__global__ __launch_bounds__(kLayouts[L].LX * kLayouts[L].LY * kLayouts[L].LZ)
__attribute__((amdgpu_waves_per_eu(kImageWaves, kImageWaves))) void reproject_kernel(
    Workspace ws, const SwathDev* __restrict__ swaths, const int* __restrict__ order,
    const int* __restrict__ tile_swath, const PingRange* __restrict__ prange, int n_tiles) {
  extern __shared__ __align__(16) unsigned char lds[];
  constexpr int K = kLayouts[L].K, LX = kLayouts[L].LX, LY = kLayouts[L].LY, LZ = kLayouts[L].LZ;
  constexpr int NT = LX * LY * LZ, NW = NT / 64;
  constexpr int TX = LX * K, TY = LY, TZ = LZ, ROWS = LY * LZ;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  // Lanes run along the pixel rows first (the image kernel runs along x):
  // pixels of one row that are close in x fall on the same echo samples, so
  // a wave spread over many rows scatters to mostly distinct LDS addresses.
  const int row = tid % ROWS, lx = tid / ROWS;
  const int ly = row % LY, lz = row / LY;
  __shared__ int s_item;
  __shared__ int s_npart;
  __shared__ float s_wmax[NW];

  for (;;) {
    __syncthreads();
    if (tid == 0) s_item = next_tile(ws, blockIdx.x % kXcds);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);
    if (item < 0) break;
    const int t = __builtin_amdgcn_readfirstlane(order[item]);
    const int s = __builtin_amdgcn_readfirstlane(tile_swath[t]);
    const SwathDev& sw = swaths[s];
    const int E = sw.E, W = sw.W, RC = sw.RC, Ns = sw.Ns;
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
    const PingRange pr = prange[t];
    const LdsLayout Ld = lds_layout(RC, chunk_pings(RC, E), W, ROWS, GATE);
    const TxRec* ltx = reinterpret_cast<const TxRec*>(lds + Ld.off_tx);
    const RxRec* lrx = reinterpret_cast<const RxRec*>(lds + Ld.off_rx);
    const int* ln0 = reinterpret_cast<const int*>(lds + Ld.off_n0);
    const int* lrows = reinterpret_cast<const int*>(lds + Ld.off_rows);
    int2* lacc = reinterpret_cast<int2*>(lds + Ld.off_win);
    const int WA = W + 2;   // accumulator entries per record

    const float sx = (float)sw.d[0], sy = (float)sw.d[1], sz = (float)sw.d[2];
    float dx[K], dsq[K], yr[K], yi[K];
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
      yr[k] = g.x;
      yi[k] = g.y;
    }
    // fixed-point scale of this tile (see the file comment)
    float m = 0.0f;
#pragma unroll
    for (int k = 0; k < K; ++k) m = fmaxf(m, fmaxf(fabsf(yr[k]), fabsf(yi[k])));
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if (lane == 0) s_wmax[wave] = m;
    __syncthreads();
    m = s_wmax[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) m = fmaxf(m, s_wmax[w]);
    if (!(m > 0.0f) || !isfinite(m)) continue;   // uniform: Y is zero (or not finite) on this tile
    const float fx_scale = 1073741824.0f / ((float)(K * NT) * m);
    const float fx_unscale = 1.0f / fx_scale;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      yr[k] *= fx_scale;
      yi[k] *= fx_scale;
    }
    const float szero = (float)W;
    const Geo geo = geo_for(ws, sw, ROWS, GATE);
    int* lpart = reinterpret_cast<int*>(lds + Ld.off_win);

    for (int P0 = pr.lo; P0 <= pr.hi; P0 += sw.SC) {
      const int sc = min(sw.SC, pr.hi - P0 + 1);
      __syncthreads();
      build_geometry<NT, TX, LY, LZ, GATE>(geo, lpart, &s_npart, ws, sw, c, C, P0, sc, x0, y0, z0, tid);
      float dT[K];
      int dT_slot = -1;
      for (int q0 = 0; q0 < sc * E; q0 += RC) {
        const int nr = min(RC, sc * E - q0);
        const int sa = q0 / E, sb = (q0 + nr - 1) / E;
        if (q0 > 0) __syncthreads();
        load_records<NT, ROWS, GATE>(lds, geo, sw, q0, nr, sa, sb - sa + 1, Ld, tid);
        for (int i = tid; i < nr * WA; i += NT) lacc[i] = make_int2(0, 0);
        __syncthreads();
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
          }
          const int r_lo = max(slot * E, q0) - q0, r_hi = min(slot * E + E, q0 + nr) - q0;
          for (int r = r_lo; r < r_hi; ++r) {
            const unsigned f = __builtin_amdgcn_readfirstlane(__float_as_uint(lrx[r].q0.w));
            if (f & kFlagSkip) continue;
            const RxRec rec = lrx[r];
            // entry n of this record's window at lds_address(lacc + r * WA) + 8 n;
            // the rounded value's bits hold n + 2^23
            const unsigned base = lds_address(lacc + (size_t)r * WA) - (kRoundMagicBits << 3);
            if (!GATE || (f & kFlagFull)) {
              if (f & kFlagDeg4)
                scatter<K, LX, 4, false>(rec, base, dx, dsq, dT, dyl, dzl, fs_c, fc_c, szero, 0, 0, yr, yi);
              else if (f & kFlagPoly)
                scatter<K, LX, 5, false>(rec, base, dx, dsq, dT, dyl, dzl, fs_c, fc_c, szero, 0, 0, yr, yi);
              else
                scatter<K, LX, 0, false>(rec, base, dx, dsq, dT, dyl, dzl, fs_c, fc_c, szero, 0, 0, yr, yi);
            } else {
              const int v = lrows[r * ROWS + row];
              const int a = row_lo(v), b = row_hi(v);
              if (f & kFlagDeg4)
                scatter<K, LX, 4, true>(rec, base, dx, dsq, dT, dyl, dzl, fs_c, fc_c, szero, lx - a, b - a, yr, yi);
              else if (f & kFlagPoly)
                scatter<K, LX, 5, true>(rec, base, dx, dsq, dT, dyl, dzl, fs_c, fc_c, szero, lx - a, b - a, yr, yi);
              else
                scatter<K, LX, 0, true>(rec, base, dx, dsq, dT, dyl, dzl, fs_c, fc_c, szero, lx - a, b - a, yr, yi);
            }
          }
        }
        __syncthreads();
        // add the chunk's windows into the output rows (samples inside the record only)
        const size_t row0 = (size_t)P0 * E + q0;
        for (int i = tid; i < nr * WA; i += NT) {
          const int r = i / WA, k = i - r * WA;
          const unsigned f = __float_as_uint(lrx[r].q0.w);
          const int n = ln0[r] + k;
          const int2 v = lacc[i];
          if (!(f & kFlagSkip) && n >= 0 && n < Ns && (v.x != 0 || v.y != 0)) {
            float* dst = reinterpret_cast<float*>(sw.gecho + (row0 + r) * (size_t)Ns + n);
            global_add(dst, (float)v.x * fx_unscale);
            global_add(dst + 1, (float)v.y * fx_unscale);
          }
        }
      }
    }
  }
}

__global__ __launch_bounds__(kThreads) void zero_rows_kernel(float2* p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = make_float2(0.0f, 0.0f);
}

// ------------------------------------------------------------ dispatch ---

typedef void (*ReprojectKernelFn)(Workspace, const SwathDev*, const int*, const int*, const PingRange*, int);

template <int L>
static ReprojectKernelFn reproject_for_layout(bool gate) {
  return gate ? reproject_kernel<L, true> : reproject_kernel<L, false>;
}

ReprojectKernelFn reproject_kernel_for(int layout, bool gate) {
  switch (layout) {
    case 0: return reproject_for_layout<0>(gate);
    case 1: return reproject_for_layout<1>(gate);
    case 2: return reproject_for_layout<2>(gate);
    case 3: return reproject_for_layout<3>(gate);
    case 4: return reproject_for_layout<4>(gate);
    case 5: return reproject_for_layout<5>(gate);
    case 6: return reproject_for_layout<6>(gate);
    case 7: return reproject_for_layout<7>(gate);
    case 8: return reproject_for_layout<8>(gate);
    default: return nullptr;
  }
}

hipError_t launch_reproject(ReprojectKernelFn fn, const Workspace& ws, int n_tiles, int grid, int threads,
                            int lds_bytes, hipStream_t st) {
  hipLaunchKernelGGL(fn, dim3(grid), dim3(threads), lds_bytes, st, ws, (const SwathDev*)ws.swaths,
                     (const int*)ws.order, (const int*)ws.tile_swath, (const PingRange*)ws.prange, n_tiles);
  return hipGetLastError();
}

hipError_t launch_zero_rows(void* p, long long n, hipStream_t st) {
  long long blocks = (n + kThreads - 1) / kThreads;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(zero_rows_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, st, reinterpret_cast<float2*>(p), n);
  return hipGetLastError();
}

hipError_t reproject_occupancy(ReprojectKernelFn fn, int threads, int lds_bytes, int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, threads, lds_bytes);
}

hipError_t set_reproject_lds_limit(ReprojectKernelFn fn, int lds_bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                             lds_bytes);
}

}  // namespace sasbp

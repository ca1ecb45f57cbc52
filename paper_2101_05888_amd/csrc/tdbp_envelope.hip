// Echo envelope for the incoherent stage of the sharpness autofocus: every
// complex sample e of a cube replaced by (|e|, 0) in the same storage format.
// Imaged with the carrier off (f_c = 0), the envelope's sharpness varies on
// the scale of the range resolution rather than the wavelength (Sec. II-A's
// delay-and-sum with the phase term removed), so a gradient ascent started
// centimetres from the track has no wrapped maxima to fall into.
//
// |e| is formed in FP32 as sqrt(re^2 + im^2) with the correctly rounded
// square root; 16-bit formats are widened to FP32 first and |e| is rounded to
// the nearest representable value (ties to even) on the way back. One thread
// per sample; HBM-bound (read and write once).
#include "tdbp_dev.h"

namespace sasbp {

__device__ __forceinline__ unsigned short float_to_bf16_rne(float x) {
  const unsigned u = __float_as_uint(x);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

template <int DT>
__global__ __launch_bounds__(kThreads) void envelope_kernel(const void* __restrict__ in, void* __restrict__ out,
                                                            long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if constexpr (DT == 0) {
    const float2 v = reinterpret_cast<const float2*>(in)[i];
    reinterpret_cast<float2*>(out)[i] = make_float2(sqrtf(fmaf(v.x, v.x, v.y * v.y)), 0.0f);
  } else if constexpr (DT == 1) {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    const h2 v = reinterpret_cast<const h2*>(in)[i];
    const float re = (float)v.x, im = (float)v.y;
    h2 o;
    o.x = (_Float16)sqrtf(fmaf(re, re, im * im));
    o.y = (_Float16)0.0f;
    reinterpret_cast<h2*>(out)[i] = o;
  } else {
    const unsigned w = reinterpret_cast<const unsigned*>(in)[i];
    const float re = __uint_as_float(w << 16), im = __uint_as_float(w & 0xffff0000u);
    reinterpret_cast<unsigned*>(out)[i] = (unsigned)float_to_bf16_rne(sqrtf(fmaf(re, re, im * im)));
  }
}

hipError_t launch_envelope(const void* in, void* out, long long n, int dt, hipStream_t st) {
  const dim3 grid((unsigned)((n + kThreads - 1) / kThreads));
  if (dt == 0) hipLaunchKernelGGL(envelope_kernel<0>, grid, dim3(kThreads), 0, st, in, out, n);
  else if (dt == 1) hipLaunchKernelGGL(envelope_kernel<1>, grid, dim3(kThreads), 0, st, in, out, n);
  else hipLaunchKernelGGL(envelope_kernel<2>, grid, dim3(kThreads), 0, st, in, out, n);
  return hipGetLastError();
}

}  // namespace sasbp

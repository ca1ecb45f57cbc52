// 4096-point complex FP32 transform for one 256-thread workgroup, in three
// radix-16 passes through LDS (used by the fused range compression).
//
// Index split (decimation in frequency): a sample index n = 256 n1 + n2 and a
// bin k = k1 + 16 k2 with n1, k1 < 16; the 256-point sub-transforms split the
// same way again. Pass 1 (thread t = n2) transforms over n1 in registers and
// applies W_4096^(n2 k1); pass 2 transforms each 256-point sub-problem over its
// leading digit and applies W_256; pass 3 finishes the 16-point transforms,
// leaving thread t with bins t + 256 j, j < 16, in natural order. The inverse
// runs the same passes with conjugate twiddles on data held that way, so a
// forward transform, a pointwise product and an inverse need no reordering.
//
// LDS holds the 4096 values at 290 a + 17 b + c for the digit triple
// (a, b, c) of 256 a + 16 b + c (17 b + c < 290, and 290 = 2 mod 32): the
// 64 lanes of passes 2 and 3 then touch each 8-byte bank pair exactly twice.
// Twiddles come from one table of kFftTw entries, rounded from FP64: pass 1's
// W^(t k1) at (k1 - 1) 256 + t and pass 2's W^(16 c j1) at 3840 + (j1 - 1) 16
// + c (k1, j1 = 1..15), W = exp(-2 pi i / 4096); the inverse conjugates them.
#pragma once

#include <hip/hip_runtime.h>

namespace sasbp {

constexpr int kFftN = 4096;
constexpr int kFftThreads = 256;
constexpr int kFftLds = 15 * 290 + 15 * 17 + 15 + 1;
constexpr int kFftTw = 15 * 256 + 15 * 16;
constexpr int kFftTw2 = 15 * 256;   // start of pass 2's twiddles

__host__ __device__ __forceinline__ int fft_lds(int a, int b, int c) { return a * 290 + b * 17 + c; }

__host__ __device__ __forceinline__ float2 fft_cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__host__ __device__ __forceinline__ float2 fft_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ float2 fft_sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// Table entry i (forward) or its conjugate (inverse)
template <bool INV>
__host__ __device__ __forceinline__ float2 fft_tw(const float2* T, int i) {
  const float2 w = T[i];
  return INV ? make_float2(w.x, -w.y) : w;
}

// The table's entry i in FP64: the exponent k of W^k it holds
__host__ __device__ __forceinline__ int fft_tw_exponent(int i) {
  return i < kFftTw2 ? (i / 256 + 1) * (i % 256) : 16 * ((i - kFftTw2) / 16 + 1) * ((i - kFftTw2) % 16);
}

// Length-4 transform in place: forward uses W_4 = -i, inverse +i.
template <bool INV>
__host__ __device__ __forceinline__ void fft_dft4(float2& x0, float2& x1, float2& x2, float2& x3) {
  const float2 s02 = fft_add(x0, x2), d02 = fft_sub(x0, x2);
  const float2 s13 = fft_add(x1, x3), d13 = fft_sub(x1, x3);
  const float2 r = INV ? make_float2(-d13.y, d13.x) : make_float2(d13.y, -d13.x);
  x0 = fft_add(s02, s13);
  x2 = fft_sub(s02, s13);
  x1 = fft_add(d02, r);
  x3 = fft_sub(d02, r);
}

// Length-16 transform in registers, natural order in and out (4 x 4 split).
template <bool INV>
__host__ __device__ __forceinline__ void fft_dft16(float2 (&v)[16]) {
  // cos and sin of 2 pi m / 16, m <= 9
  constexpr float C[10] = {1.0f, 0.923879533f, 0.707106781f, 0.382683432f, 0.0f,
                           -0.382683432f, -0.707106781f, -0.923879533f, -1.0f, -0.923879533f};
  constexpr float S[10] = {0.0f, 0.382683432f, 0.707106781f, 0.923879533f, 1.0f,
                           0.923879533f, 0.707106781f, 0.382683432f, 0.0f, -0.382683432f};
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) fft_dft4<INV>(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
#pragma unroll
  for (int k1 = 1; k1 < 4; ++k1)
#pragma unroll
    for (int n2 = 1; n2 < 4; ++n2) {
      const int m = n2 * k1;
      v[4 * k1 + n2] = fft_cmul(v[4 * k1 + n2], make_float2(C[m], INV ? S[m] : -S[m]));
    }
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) fft_dft4<INV>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
  float2 t[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) t[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = t[i];
}

// Pass 1: thread t holds x[256 n1 + t] in v[n1]; transforms, applies the
// twiddles and stores. The caller synchronises before the store when LDS may
// still be read.
template <bool INV>
__host__ __device__ __forceinline__ void fft_pass1_compute(float2 (&v)[16], int t, const float2* T) {
  fft_dft16<INV>(v);
#pragma unroll
  for (int k1 = 1; k1 < 16; ++k1) v[k1] = fft_cmul(v[k1], fft_tw<INV>(T, (k1 - 1) * 256 + t));
}

__host__ __device__ __forceinline__ void fft_pass1_store(const float2 (&v)[16], int t, float2* A) {
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) A[fft_lds(k1, t >> 4, t & 15)] = v[k1];
}

// Pass 2: thread t owns the 16 slots (a, *, c) with a = t & 15, c = t >> 4.
template <bool INV>
__host__ __device__ __forceinline__ void fft_pass2(int t, const float2* T, float2* A) {
  const int a = t & 15, c = t >> 4;
  float2 v[16];
#pragma unroll
  for (int m1 = 0; m1 < 16; ++m1) v[m1] = A[fft_lds(a, m1, c)];
  fft_dft16<INV>(v);
#pragma unroll
  for (int j1 = 1; j1 < 16; ++j1) v[j1] = fft_cmul(v[j1], fft_tw<INV>(T, kFftTw2 + (j1 - 1) * 16 + c));
#pragma unroll
  for (int j1 = 0; j1 < 16; ++j1) A[fft_lds(a, j1, c)] = v[j1];
}

// Pass 3: thread t = a + 16 b ends with bin t + 256 j in v[j].
template <bool INV>
__host__ __device__ __forceinline__ void fft_pass3(float2 (&v)[16], int t, const float2* A) {
  const int a = t & 15, b = t >> 4;
#pragma unroll
  for (int m2 = 0; m2 < 16; ++m2) v[m2] = A[fft_lds(a, b, m2)];
  fft_dft16<INV>(v);
}

}  // namespace sasbp

// Complex arithmetic on float2 (x = real, y = imaginary) for the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace cs {

__device__ __forceinline__ float2 c2(float re, float im) { return make_float2(re, im); }
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return c2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return c2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return c2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cconj(float2 a) { return c2(a.x, -a.y); }
// a * b
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return c2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return c2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -a.x * b.y));
}
// conj(a) * b
__device__ __forceinline__ float2 cconjmul(float2 a, float2 b) {
  return c2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.x, b.y, -a.y * b.x));
}
// i * a
__device__ __forceinline__ float2 cmuli(float2 a) { return c2(-a.y, a.x); }
// -i * a
__device__ __forceinline__ float2 cmulmi(float2 a) { return c2(a.y, -a.x); }
__device__ __forceinline__ float cabs2(float2 a) { return fmaf(a.x, a.x, a.y * a.y); }

// Soft threshold of Eq. 4 with a strict comparison: |v| == g maps to 0.
__device__ __forceinline__ float soft(float v, float g) {
  const float a = fabsf(v) - g;
  return a > 0.0f ? copysignf(a, v) : 0.0f;
}

}  // namespace cs

// MFMA traits shared by the kernels (gfx950).  A 16x16x4 MFMA takes A[i][k]
// from lane i + 16k and B[k][j] from lane j + 16k; element r of the result
// holds row MF<T>::row(lane, r), column lane & 15 (the f32 and f64
// instructions place rows differently; measured on gfx950).
#pragma once
#include <hip/hip_runtime.h>

namespace mpo {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

template <typename T> struct MF;
template <> struct MF<float> {
  typedef v4f acc;
  __device__ static acc mma(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <> struct MF<double> {
  typedef v4d acc;
  __device__ static acc mma(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

}  // namespace mpo

namespace mpo {

// Split-BF16 products on v_mfma_f32_16x16x32_bf16: x = hi + lo with
// hi = bf16(x), lo = bf16(x - hi); a*b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi
// (the lo*lo term is below 2^-16 relative), accumulated in FP32.  Lane l
// supplies A[l & 15][8 (l >> 4) + e] and B[8 (l >> 4) + e][l & 15], e < 8; the
// result layout is that of the f32 16x16x4 instruction (measured on gfx950).
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

struct Split8 {
  v8bf hi, lo;
};

__device__ __forceinline__ void split_set(Split8& s, int e, float x) {
  const __bf16 h = (__bf16)x;
  s.hi[e] = h;
  s.lo[e] = (__bf16)(x - (float)h);
}

__device__ __forceinline__ v4f mma3_bf16(const Split8& a, const Split8& b, v4f c) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.lo, b.hi, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.lo, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.hi, c, 0, 0, 0);
  return c;
}

}  // namespace mpo

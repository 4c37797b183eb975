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

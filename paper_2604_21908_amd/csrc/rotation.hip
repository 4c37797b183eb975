// Panel rotation of the block one-sided Jacobi SVD (gfx950): P <- P + P D
// for the 32-column panels of a round-robin step, D = W - I from the panel
// EVD (jacobi.hip), over row chunks (a launch argument) of theta's operand and of the
// accumulated rotations V.
//
//   k_jac_rot        FP MFMA (f32 16x16x4 or f64 16x16x4), computed as
//                    P^T <- P^T + D^T P^T so that each 16-lane group of a wave
//                    reads and writes 16 consecutive rows of one column
//   k_jac_rot_mixed  the mixed form in one launch: theta's row chunks on
//                    split-BF16 products, V's on FP32 MFMA
#include "common.h"
#include "mfma.h"

namespace mpo {

// ---------------------------------------------------------------- rotation
// Row space of a panel: rows [0, m) of theta's operand A, then rows [0, nv)
// of V.  out^T = P^T + D^T P^T for 16-row strips; lane (l & 15) owns row
// strip0 + (l & 15).
// part 0: all rows; 1: theta's rows [0, m) only; 2: V's rows only.
// Element (row rho, panel column c) of the panel's row space: rows [0, m) of
// theta's operand A, then V's rows.
template <typename T>
__device__ __forceinline__ cx<T>* panel_ptr(const JacProb& P, int bi, int bj, int rho, int c) {
  if (rho < P.m) return (cx<T>*)P.A + (size_t)panel_col(bi, bj, c) * P.lda + rho;
  return (cx<T>*)P.V + (size_t)panel_col(bi, bj, c) * P.ncol_pad + (rho - P.m);
}

// A wave's 16-row strip is loaded once, element (row lane & 15, column
// (lane >> 4) + 4 u) into slot u -- the MFMA B-operand layout, 16 consecutive
// rows of a column per 16-lane group -- with rows past c1 clamped to a valid
// row (never stored).  The accumulator layout is read back through the wave's
// own LDS tile.  DS instructions of one wave execute in order, so the tile
// needs no barrier; the wave_barrier only keeps the compiler from reordering.
template <typename T>
struct StripBase {
  cx<T>* base;   // A or V
  int ld;
  int row;       // clamped row within base
};
template <typename T>
__device__ __forceinline__ StripBase<T> strip_base(const JacProb& P, int rho) {
  if (rho < P.m) return StripBase<T>{(cx<T>*)P.A, P.lda, rho};
  return StripBase<T>{(cx<T>*)P.V, P.ncol_pad, rho - P.m};
}
// colB[u]: panel column of load slot u; colA[4 t + r]: of accumulator entry
template <typename T>
__device__ __forceinline__ void strip_load(const StripBase<T>& sb, const int (&colB)[8], cx<T> (&v)[8]) {
#pragma unroll
  for (int u = 0; u < 8; ++u) v[u] = sb.base[colB[u] * sb.ld + sb.row];   // < 2^24 elements: int offsets
}

// Rows [c0, c1) of the panel's row space, FP MFMA (T = float or double).
// Software-pipelined: a wave issues the loads of its next strip before it
// multiplies and stores the current one.
template <typename T>
__device__ __forceinline__ void rot_rows(const JacProb& P, int bi, int bj, int c0, int c1, const cx<T> (*Ds)[33],
                                         cx<T> (*Sw)[33]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  typedef typename MF<T>::acc acc_t;
  int colB[8], colA[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) colB[u] = panel_col(bi, bj, (lane >> 4) + 4 * u);
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) colA[4 * t + r] = panel_col(bi, bj, t * 16 + MF<T>::row(lane, r));
  int s0 = c0 + wave * 16;
  if (s0 >= c1) return;
  cx<T> v[8];
  strip_load<T>(strip_base<T>(P, min(s0 + (lane & 15), c1 - 1)), colB, v);
  for (; s0 < c1; s0 += 64) {
    const bool more = s0 + 64 < c1;
    cx<T> nv[8];
    if (more) strip_load<T>(strip_base<T>(P, min(s0 + 64 + (lane & 15), c1 - 1)), colB, nv);
#pragma unroll
    for (int u = 0; u < 8; ++u) Sw[lane & 15][(lane >> 4) + 4 * u] = v[u];
    __builtin_amdgcn_wave_barrier();
    T pre[2][4], pim[2][4];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const cx<T> a = Sw[lane & 15][t * 16 + MF<T>::row(lane, r)];
        pre[t][r] = a.re;
        pim[t][r] = a.im;
      }
    __builtin_amdgcn_wave_barrier();
    // The increment P D as three real products (Gauss): with D = Dr + i Di and
    // P = Pr + i Pi, t1 = Dr Pr, t2 = Di Pi, t3 = (Dr + Di)(Pr + Pi), then
    // Re = t1 - t2 and Im = t3 - t1 - t2 -- three MFMA chains instead of four.
    // The increment is formed on its own and only then added to P, so no
    // product is taken of P's own (large) values.
    acc_t t1[2], t2[2], t3[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) t1[t] = t2[t] = t3[t] = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      const int k = 4 * kk + (lane >> 4);
      const cx<T> x = v[kk];
      const T xs = x.re + x.im;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const cx<T> d = Ds[k][t * 16 + (lane & 15)];   // A[c][k] = D[k][c]
        t1[t] = MF<T>::mma(d.re, x.re, t1[t]);
        t2[t] = MF<T>::mma(d.im, x.im, t2[t]);
        t3[t] = MF<T>::mma(d.re + d.im, xs, t3[t]);
      }
    }
    const int rho = s0 + (lane & 15);
    if (rho < c1) {
      const StripBase<T> sb = strip_base<T>(P, rho);
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          sb.base[colA[4 * t + r] * sb.ld + sb.row] =
              cx<T>{pre[t][r] + (t1[t][r] - t2[t][r]), pim[t][r] + ((t3[t][r] - t1[t][r]) - t2[t][r])};
    }
    if (more) {
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = nv[u];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_jac_rot(JacBatch jb, int step, int part, int rrc) {
  const int pi = blockIdx.z;
  if (pi >= jb.count) return;
  const JacProb P = jb.p[pi];
  if (step >= P.nblk - 1 || (int)blockIdx.x >= P.nblk / 2) return;
  if (P.st->active == 0) return;
  if (P.pflag[blockIdx.x] == 0) return;
  const int nv = P.V ? P.ncol : 0;
  const int rows = (part == 1) ? P.m : P.m + nv;
  const int c0 = (part == 2 ? P.m : 0) + blockIdx.y * rrc;
  if (c0 >= rows) return;
  const int c1 = min(rows, c0 + rrc);
  int bi, bj;
  rr_pair2(P.nblk, step, blockIdx.x, bi, bj);
  __shared__ cx<T> Ds[32][33];
  __shared__ cx<T> Sw[4][16][33];   // one strip tile per wave
  const cx<T>* D = (const cx<T>*)P.dmat + (size_t)blockIdx.x * 1024;
  for (int e = threadIdx.x; e < 1024; e += 256) Ds[e >> 5][e & 31] = D[e];
  __syncthreads();
  rot_rows<T>(P, bi, bj, c0, c1, Ds, Sw[threadIdx.x >> 6]);
}

// ---------------------------------------------------------------- split-BF16
// theta's rows [c0, c1) (c1 <= m) on split-BF16 products; the accumulated
// rotations V stay on FP32 MFMA (rot_rows) so that V remains unitary to FP32
// accuracy.
__device__ __forceinline__ void rot_rows_bf16(const JacProb& P, int bi, int bj, int c0, int c1,
                                              const cx<float> (*Ds)[33], cx<float> (*Sw)[33]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g8 = (lane >> 4) * 8;
  // A operands D^T[c][k] = D[k][c] for the two 16-column halves, split once
  Split8 dr[2], di[2], dn[2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const cx<float> d = Ds[g8 + e][t * 16 + (lane & 15)];
      split_set(dr[t], e, d.re);
      split_set(di[t], e, d.im);
      split_set(dn[t], e, -d.im);
    }
  int colB[8], colA[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) colB[u] = panel_col(bi, bj, (lane >> 4) + 4 * u) * P.lda;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) colA[4 * t + r] = panel_col(bi, bj, t * 16 + MF<float>::row(lane, r)) * P.lda;
  const cx<float>* A = (const cx<float>*)P.A;
  cx<float>* Aw = (cx<float>*)P.A;
  int s0 = c0 + wave * 16;
  if (s0 >= c1) return;
  cx<float> v[8];
  {
    const int row = min(s0 + (lane & 15), c1 - 1);
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = A[colB[u] + row];
  }
  for (; s0 < c1; s0 += 64) {
    const bool more = s0 + 64 < c1;
    cx<float> nv[8];
    if (more) {
      const int row = min(s0 + 64 + (lane & 15), c1 - 1);
#pragma unroll
      for (int u = 0; u < 8; ++u) nv[u] = A[colB[u] + row];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) Sw[lane & 15][(lane >> 4) + 4 * u] = v[u];
    __builtin_amdgcn_wave_barrier();
    v4f cre[2], cim[2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const cx<float> a = Sw[lane & 15][t * 16 + MF<float>::row(lane, r)];
        cre[t][r] = a.re;
        cim[t][r] = a.im;
      }
    Split8 xr, xi;   // B operand: this lane's columns g8 .. g8 + 7
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const cx<float> x = Sw[lane & 15][g8 + e];
      split_set(xr, e, x.re);
      split_set(xi, e, x.im);
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      cre[t] = mma3_bf16(dr[t], xr, cre[t]);
      cre[t] = mma3_bf16(dn[t], xi, cre[t]);
      cim[t] = mma3_bf16(dr[t], xi, cim[t]);
      cim[t] = mma3_bf16(di[t], xr, cim[t]);
    }
    const int row = s0 + (lane & 15);
    if (row < c1) {
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) Aw[colA[4 * t + r] + row] = cx<float>{cre[t][r], cim[t][r]};
    }
    if (more) {
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = nv[u];
    }
  }
}

// One launch for both row sets of the mixed form: row chunks y < ny_theta
// rotate theta's rows on split-BF16, the others V's rows on FP32, so the
// memory-bound and the MFMA-bound workgroups share the machine.
__global__ __launch_bounds__(256) void k_jac_rot_mixed(JacBatch jb, int step, int ny_theta, int rrc) {
  const int pi = blockIdx.z;
  if (pi >= jb.count) return;
  const JacProb P = jb.p[pi];
  if (step >= P.nblk - 1 || (int)blockIdx.x >= P.nblk / 2) return;
  if (P.st->active == 0) return;
  if (P.pflag[blockIdx.x] == 0) return;
  const bool theta = (int)blockIdx.y < ny_theta;
  int c0, c1;
  if (theta) {
    c0 = blockIdx.y * rrc;
    if (c0 >= P.m) return;
    c1 = min(P.m, c0 + rrc);
  } else {
    const int nv = P.V ? P.ncol : 0;
    c0 = P.m + (blockIdx.y - ny_theta) * rrc;
    if (c0 >= P.m + nv) return;
    c1 = min(P.m + nv, c0 + rrc);
  }
  int bi, bj;
  rr_pair2(P.nblk, step, blockIdx.x, bi, bj);
  __shared__ cx<float> Ds[32][33];
  __shared__ cx<float> Sw[4][16][33];   // one strip tile per wave
  const cx<float>* D = (const cx<float>*)P.dmat + (size_t)blockIdx.x * 1024;
  for (int e = threadIdx.x; e < 1024; e += 256) Ds[e >> 5][e & 31] = D[e];
  __syncthreads();
  if (theta) rot_rows_bf16(P, bi, bj, c0, c1, Ds, Sw[threadIdx.x >> 6]);
  else rot_rows<float>(P, bi, bj, c0, c1, Ds, Sw[threadIdx.x >> 6]);
}

// Row chunks of rrc rows (a multiple of 64: four waves of 16-row strips):
// maxrch_a chunks of theta's rows, then maxrch_v of V's.
template <typename T>
void launch_jac_rot(const JacBatch& b, int maxpairs, int maxrch_a, int maxrch_v, int step, int mode, int rrc,
                    hipStream_t s) {
  if (mode == ROT_MIXED)
    hipLaunchKernelGGL(k_jac_rot_mixed, dim3(maxpairs, maxrch_a + maxrch_v, b.count), dim3(256), 0, s, b, step,
                       maxrch_a, rrc);
  else
    hipLaunchKernelGGL(k_jac_rot<T>, dim3(maxpairs, maxrch_a + maxrch_v, b.count), dim3(256), 0, s, b, step, 0,
                       rrc);
}
template <>
void launch_jac_rot<double>(const JacBatch& b, int maxpairs, int maxrch_a, int maxrch_v, int step, int, int rrc,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_jac_rot<double>, dim3(maxpairs, maxrch_a + maxrch_v, b.count), dim3(256), 0, s, b, step, 0,
                     rrc);
}
template void launch_jac_rot<float>(const JacBatch&, int, int, int, int, int, int, hipStream_t);

}  // namespace mpo

// Householder QR preconditioner of the Jacobi SVD (gfx950).
//
// The bond matrix enters as M = (lambda theta)^dag, n x m column-major.  Its
// QR factorisation M = Q R gives theta = L Q^dag with L = R^dag lower
// trapezoidal; one-sided Jacobi on the columns of L then needs far fewer
// sweeps than on theta itself (the QR-preconditioned Jacobi SVD of Drmac and
// Veselic), and the right singular vectors of theta are V = Q [W; 0] with W
// the accumulated Jacobi rotations -- no division by singular values.
//
//   k_qr_panel   one workgroup factors a QNB-column panel (complex Householder
//                reflectors, LAPACK's sign convention) and builds the
//                upper-triangular T of the compact WY form; FP64 reductions
//   k_qr_apply   C <- (I - V op(T) V^dag) C on 16-column tiles: the trailing
//                update (op = dag) and the formation of V (op = identity)
//   k_lower_from_r  L = R^dag into the column-major Jacobi operand
//   k_build_y / k_vh_rows   [W_k; 0] and B_{i+1} <- V_k^dag, lambda_i <- s_<k
#include "common.h"
#include "mfma.h"

namespace mpo {

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename T>
__global__ __launch_bounds__(1024) void k_qr_panel(QrBatch qb, int p0) {
  const int pi = blockIdx.x;
  if (pi >= qb.count) return;
  const QrProb P = qb.p[pi];
  if (p0 >= P.r) return;
  const int nb = min(QNB, P.r - p0);
  const int n = P.n;
  cx<T>* M = (cx<T>*)P.M;
  cx<T>* tau = (cx<T>*)P.tau;
  cx<T>* Tf = (cx<T>*)P.Tf + (size_t)(p0 / QNB) * QNB * QNB;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  __shared__ double red[16][2 * QNB];
  __shared__ double res[2 * QNB];
  __shared__ double bc[8];
  __shared__ cx<double> Tl[QNB][QNB];

  for (int jj = 0; jj < nb; ++jj) {
    const int j = p0 + jj;
    cx<T>* colj = M + (size_t)j * n;
    // |x[j+1:n]|^2
    double s = 0;
    for (int i = j + 1 + tid; i < n; i += 1024) {
      const double a = colj[i].re, b = colj[i].im;
      s += a * a + b * b;
    }
    s = wave_sum(s);
    if (lane == 0) red[wv][0] = s;
    __syncthreads();
    if (tid == 0) {
      double xn2 = 0;
      for (int w = 0; w < 16; ++w) xn2 += red[w][0];
      const double ar = colj[j].re, ai = colj[j].im;
      double tr = 0, ti = 0, scr = 0, sci = 0, beta = ar;
      if (xn2 > 0 || ai != 0) {
        const double nrm = sqrt(ar * ar + ai * ai + xn2);
        beta = (ar >= 0) ? -nrm : nrm;
        tr = (beta - ar) / beta;
        ti = -ai / beta;
        const double dr = ar - beta, di = ai, d2 = dr * dr + di * di;
        scr = dr / d2;
        sci = -di / d2;
      } else {
        beta = ar;
      }
      bc[0] = beta;
      bc[1] = tr;
      bc[2] = ti;
      bc[3] = scr;
      bc[4] = sci;
    }
    __syncthreads();
    const double beta = bc[0], tr = bc[1], ti = bc[2], scr = bc[3], sci = bc[4];
    const bool trivial = (tr == 0.0 && ti == 0.0);
    if (!trivial)
      for (int i = j + 1 + tid; i < n; i += 1024) {
        const double a = colj[i].re, b = colj[i].im;
        colj[i] = cx<T>{(T)(a * scr - b * sci), (T)(a * sci + b * scr)};
      }
    __syncthreads();
    if (tid == 0) {
      colj[j] = cx<T>{(T)beta, (T)0};
      tau[j] = cx<T>{(T)tr, (T)ti};
    }
    // dots over rows >= j: slot q < jj -> z_q = v_q^dag v_j (for T);
    //                      slot q >= jj -> w = v_j^dag M[:, p0+q+1] (update)
    const int nd = nb - 1;
    double acc[2 * (QNB - 1)];
#pragma unroll
    for (int q = 0; q < 2 * (QNB - 1); ++q) acc[q] = 0;
    for (int i = j + tid; i < n; i += 1024) {
      const cx<T> vt = colj[i];
      const double vr = (i == j) ? 1.0 : (double)vt.re, vi = (i == j) ? 0.0 : (double)vt.im;
#pragma unroll
      for (int q = 0; q < QNB - 1; ++q) {
        if (q < nd) {
          if (q < jj) {
            const cx<T> y = M[(size_t)(p0 + q) * n + i];
            acc[2 * q] += (double)y.re * vr + (double)y.im * vi;
            acc[2 * q + 1] += (double)y.re * vi - (double)y.im * vr;
          } else {
            const cx<T> y = M[(size_t)(p0 + q + 1) * n + i];
            acc[2 * q] += vr * (double)y.re + vi * (double)y.im;
            acc[2 * q + 1] += vr * (double)y.im - vi * (double)y.re;
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 2 * (QNB - 1); ++q) {
      const double v = wave_sum(acc[q]);
      if (lane == 0) red[wv][q] = v;
    }
    __syncthreads();
    if (tid < 2 * (QNB - 1)) {
      double v = 0;
      for (int w = 0; w < 16; ++w) v += red[w][tid];
      res[tid] = v;
    }
    __syncthreads();
    // later columns: M[i][c] -= conj(tau) v_i w_c, rows i >= j
    if (!trivial) {
      const double ctr = tr, cti = -ti;
      for (int q = jj; q < nd; ++q) {
        const int c = p0 + q + 1;
        const double wr = res[2 * q], wi = res[2 * q + 1];
        const double fr = ctr * wr - cti * wi, fi = ctr * wi + cti * wr;
        cx<T>* colc = M + (size_t)c * n;
        for (int i = j + tid; i < n; i += 1024) {
          const cx<T> vt = colj[i];
          const double vr = (i == j) ? 1.0 : (double)vt.re, vi = (i == j) ? 0.0 : (double)vt.im;
          const double ur = vr * fr - vi * fi, ui = vr * fi + vi * fr;
          const cx<T> x = colc[i];
          colc[i] = cx<T>{(T)((double)x.re - ur), (T)((double)x.im - ui)};
        }
      }
    }
    // T[0:jj, jj] = -tau_j T[0:jj, 0:jj] z,  T[jj][jj] = tau_j
    if (tid == 0) {
      for (int a = 0; a < jj; ++a) {
        double sr = 0, si = 0;
        for (int b = a; b < jj; ++b) {
          const cx<double> t = Tl[a][b];
          const double zr = res[2 * b], zi = res[2 * b + 1];
          sr += t.re * zr - t.im * zi;
          si += t.re * zi + t.im * zr;
        }
        Tl[a][jj] = cx<double>{-(tr * sr - ti * si), -(tr * si + ti * sr)};
      }
      Tl[jj][jj] = cx<double>{tr, ti};
      for (int a = jj + 1; a < QNB; ++a) Tl[a][jj] = cx<double>{0, 0};
    }
    __syncthreads();
  }
  if (tid < QNB * QNB) {
    const int a = tid / QNB, b = tid % QNB;
    const cx<double> t = (a < nb && b < nb && a <= b) ? Tl[a][b] : cx<double>{0, 0};
    Tf[tid] = cx<T>{(T)t.re, (T)t.im};
  }
}

// 16-column tile of C per workgroup (4 waves).  Phase 1: W1 = V^dag C over
// rows [p0, n) on MFMA from LDS-staged 64-row slabs, one K range per wave,
// then a cross-wave sum.  Phase 2: W2 = op(T) W1 (16 x 16, FP64), then
// C^T <- C^T - W2^T V^T on MFMA with each 16-lane group on 16 consecutive
// rows of one column of C.
template <typename T>
__global__ __launch_bounds__(256) void k_qr_apply(QrApplyBatch ab, int p0) {
  const int pi = blockIdx.y;
  if (pi >= ab.count) return;
  const QrApplyProb P = ab.p[pi];
  if (p0 >= P.r) return;
  const int cbeg = P.c0 + blockIdx.x * QAT;
  if (cbeg >= P.c1) return;
  const int nb = min(QNB, P.r - p0);
  const int ncols = min(QAT, P.c1 - cbeg);
  const int n = P.n;
  const cx<T>* M = (const cx<T>*)P.M;
  cx<T>* C = (cx<T>*)P.C;
  const cx<T>* Tf = (const cx<T>*)P.Tf + (size_t)(p0 / QNB) * QNB * QNB;
  typedef typename MF<T>::acc acc_t;
  __shared__ cx<T> Vs[64][QNB + 1];
  __shared__ cx<T> Cs[64][QAT + 1];
  __shared__ double Wp[4][QNB][QAT][2];
  __shared__ cx<double> W1[QNB][QAT + 1];
  __shared__ cx<T> W2[QNB][QAT + 1];
  __shared__ cx<double> Tl[QNB][QNB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  {
    const int a = tid / QNB, b = tid % QNB;
    if (ab.conj_t) {
      const cx<T> u = Tf[b * QNB + a];
      Tl[a][b] = cx<double>{(double)u.re, -(double)u.im};
    } else {
      const cx<T> t = Tf[a * QNB + b];
      Tl[a][b] = cx<double>{(double)t.re, (double)t.im};
    }
  }
  // ---- phase 1: W1[a][c] = sum_i conj(V[i][a]) C[i][c]
  acc_t wre = {0, 0, 0, 0}, wim = {0, 0, 0, 0};
  for (int r0 = p0; r0 < n; r0 += 64) {
    for (int e = tid; e < 64 * QNB; e += 256) {
      const int rr = e % 64, a = e / 64, i = r0 + rr;
      cx<T> v = {0, 0};
      if (i < n && a < nb) {
        if (i == p0 + a) v = cx<T>{1, 0};
        else if (i > p0 + a) v = M[(size_t)(p0 + a) * n + i];
      }
      Vs[rr][a] = v;
    }
    for (int e = tid; e < 64 * QAT; e += 256) {
      const int rr = e % 64, c = e / 64, i = r0 + rr;
      cx<T> v = {0, 0};
      if (i < n && c < ncols) v = C[(size_t)(cbeg + c) * P.ldc + i];
      Cs[rr][c] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = wave * 16; kk < wave * 16 + 16; kk += 4) {
      const cx<T> x = Vs[kk + (lane >> 4)][lane & 15];   // A[a][k] = conj(V[k][a])
      const cx<T> y = Cs[kk + (lane >> 4)][lane & 15];   // B[k][c] = C[k][c]
      wre = MF<T>::mma(x.re, y.re, wre);
      wre = MF<T>::mma(x.im, y.im, wre);
      wim = MF<T>::mma(x.re, y.im, wim);
      wim = MF<T>::mma(-x.im, y.re, wim);
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int a = MF<T>::row(lane, r), c = lane & 15;
    Wp[wave][a][c][0] = (double)wre[r];
    Wp[wave][a][c][1] = (double)wim[r];
  }
  __syncthreads();
  {
    const int a = tid / QAT, c = tid % QAT;
    W1[a][c] = cx<double>{Wp[0][a][c][0] + Wp[1][a][c][0] + Wp[2][a][c][0] + Wp[3][a][c][0],
                          Wp[0][a][c][1] + Wp[1][a][c][1] + Wp[2][a][c][1] + Wp[3][a][c][1]};
  }
  __syncthreads();
  {
    const int a = tid / QAT, c = tid % QAT;
    double yr = 0, yi = 0;
    for (int b = 0; b < QNB; ++b) {
      const cx<double> t = Tl[a][b], u = W1[b][c];
      yr += t.re * u.re - t.im * u.im;
      yi += t.re * u.im + t.im * u.re;
    }
    W2[a][c] = cx<T>{(T)yr, (T)yi};
  }
  __syncthreads();
  // ---- phase 2: C^T[c][i] -= sum_a W2[a][c] V[i][a], 16-row strips per wave
  for (int s0 = p0 + wave * 16; s0 < n; s0 += 64) {
    const int i = s0 + (lane & 15);
    const bool valid = i < n;
    acc_t cre, cim;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = MF<T>::row(lane, r);
      cx<T> v = {0, 0};
      if (valid && c < ncols) v = C[(size_t)(cbeg + c) * P.ldc + i];
      cre[r] = v.re;
      cim[r] = v.im;
    }
#pragma unroll
    for (int k0 = 0; k0 < QNB; k0 += 4) {
      const int a = k0 + (lane >> 4);
      cx<T> v = {0, 0};
      if (valid && a < nb) {
        if (i == p0 + a) v = cx<T>{1, 0};
        else if (i > p0 + a) v = M[(size_t)(p0 + a) * n + i];
      }
      const cx<T> w = W2[a][lane & 15];   // A[c][a] = W2[a][c], negated for the subtraction
      cre = MF<T>::mma(-w.re, v.re, cre);
      cre = MF<T>::mma(w.im, v.im, cre);
      cim = MF<T>::mma(-w.re, v.im, cim);
      cim = MF<T>::mma(-w.im, v.re, cim);
    }
    if (valid) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = MF<T>::row(lane, r);
        if (c < ncols) C[(size_t)(cbeg + c) * P.ldc + i] = cx<T>{cre[r], cim[r]};
      }
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_lower_from_r(LowerBatch lb) {
  const int pi = blockIdx.z;
  if (pi >= lb.count) return;
  const LowerProb P = lb.p[pi];
  const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
  if (i0 >= P.m || j0 >= P.rpad) return;
  __shared__ cx<T> tile[32][33];
  const cx<T>* M = (const cx<T>*)P.M;
  cx<T>* A = (cx<T>*)P.A;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int i = i0 + k, j = j0 + tx;   // read M column i (contiguous in j)
    cx<T> v = {0, 0};
    if (i < P.m && j < P.r && i >= j) {
      const cx<T> x = M[(size_t)i * P.n + j];
      v = cx<T>{x.re, -x.im};
    }
    tile[k][tx] = v;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int j = j0 + k, i = i0 + tx;   // write A column j (contiguous in i)
    if (j < P.rpad && i < P.m) A[(size_t)j * P.lda + i] = tile[tx][k];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_build_y(VkBatch vb) {
  const int pi = blockIdx.y;
  if (pi >= vb.count) return;
  const VkProb P = vb.p[pi];
  const cx<T>* W = (const cx<T>*)P.W;
  cx<T>* Y = (cx<T>*)P.Y;
  const size_t tot = (size_t)P.k * P.n;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (size_t)gridDim.x * 256) {
    const int j = (int)(e / P.n), i = (int)(e - (size_t)j * P.n);
    Y[e] = (i < P.r) ? W[(size_t)P.perm[j] * P.ldw + i] : cx<T>{0, 0};
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_vh_rows(VkBatch vb) {
  const int pi = blockIdx.y;
  if (pi >= vb.count) return;
  const VkProb P = vb.p[pi];
  const cx<T>* Y = (const cx<T>*)P.Y;
  cx<T>* R = (cx<T>*)P.right;
  const size_t tot = (size_t)P.k * P.n;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (size_t)gridDim.x * 256) {
    const cx<T> y = Y[e];
    R[e] = cx<T>{y.re, -y.im};
    const int j = (int)(e / P.n);
    if (e - (size_t)j * P.n == 0) P.lam[j] = P.s_sorted[j];
  }
}

// ---------------------------------------------------------------- launchers
template <typename T>
void launch_qr_panel(const QrBatch& b, int p0, hipStream_t s) {
  hipLaunchKernelGGL(k_qr_panel<T>, dim3(b.count), dim3(1024), 0, s, b, p0);
}
template <typename T>
void launch_qr_apply(const QrApplyBatch& b, int p0, int maxcols, hipStream_t s) {
  const int gx = (maxcols + QAT - 1) / QAT;
  if (gx < 1) return;
  hipLaunchKernelGGL(k_qr_apply<T>, dim3(gx, b.count), dim3(256), 0, s, b, p0);
}
template <typename T>
void launch_lower_from_r(const LowerBatch& b, int maxm, int maxrpad, hipStream_t s) {
  hipLaunchKernelGGL(k_lower_from_r<T>, dim3((maxm + 31) / 32, (maxrpad + 31) / 32, b.count), dim3(256), 0, s, b);
}
template <typename T>
void launch_build_y(const VkBatch& b, size_t maxel, hipStream_t s) {
  size_t g = (maxel + 255) / 256;
  g = g < 1 ? 1 : (g > 1024 ? 1024 : g);
  hipLaunchKernelGGL(k_build_y<T>, dim3((unsigned)g, b.count), dim3(256), 0, s, b);
}
template <typename T>
void launch_vh_rows(const VkBatch& b, size_t maxel, hipStream_t s) {
  size_t g = (maxel + 255) / 256;
  g = g < 1 ? 1 : (g > 1024 ? 1024 : g);
  hipLaunchKernelGGL(k_vh_rows<T>, dim3((unsigned)g, b.count), dim3(256), 0, s, b);
}

#define QINST(T)                                                                  \
  template void launch_qr_panel<T>(const QrBatch&, int, hipStream_t);             \
  template void launch_qr_apply<T>(const QrApplyBatch&, int, int, hipStream_t);   \
  template void launch_lower_from_r<T>(const LowerBatch&, int, int, hipStream_t); \
  template void launch_build_y<T>(const VkBatch&, size_t, hipStream_t);           \
  template void launch_vh_rows<T>(const VkBatch&, size_t, hipStream_t);
QINST(float)
QINST(double)

}  // namespace mpo

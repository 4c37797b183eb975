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
//   k_qr_apply   C <- (I - V op(T) V^dag) C on 32-column tiles: the trailing
//                update (op = dag) and the formation of V (op = identity)
//   k_lower_from_r  L = R^dag into the column-major Jacobi operand
//   k_build_y / k_vh_rows   [W_k; 0] and B_{i+1} <- V_k^dag, lambda_i <- s_<k
#include "common.h"

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

template <typename T>
__global__ __launch_bounds__(256) void k_qr_apply(QrApplyBatch ab, int p0) {
  const int pi = blockIdx.y;
  if (pi >= ab.count) return;
  const QrApplyProb P = ab.p[pi];
  if (p0 >= P.r) return;
  const int cbeg = P.c0 + blockIdx.x * 32;
  if (cbeg >= P.c1) return;
  const int nb = min(QNB, P.r - p0);
  const int ncols = min(32, P.c1 - cbeg);
  const int n = P.n;
  const cx<T>* M = (const cx<T>*)P.M;
  cx<T>* C = (cx<T>*)P.C;
  const cx<T>* Tf = (const cx<T>*)P.Tf + (size_t)(p0 / QNB) * QNB * QNB;
  __shared__ cx<T> Vs[64][QNB + 1];
  __shared__ cx<T> Cs[64][33];
  __shared__ cx<double> W1[QNB][33];
  __shared__ cx<double> Tl[QNB][QNB];
  const int tid = threadIdx.x;
  {
    const int a = tid / QNB, b = tid % QNB;
    const cx<T> t = Tf[a * QNB + b];
    // op(T)[a][b]: T or T^dag
    if (ab.conj_t) {
      const cx<T> u = Tf[b * QNB + a];
      Tl[a][b] = cx<double>{(double)u.re, -(double)u.im};
    } else {
      Tl[a][b] = cx<double>{(double)t.re, (double)t.im};
    }
  }
  // W1 = V^dag C over rows p0..n-1; thread -> (a = tid / 16, cols 2*(tid % 16) + {0, 1})
  const int wa = tid >> 4, wc = (tid & 15) * 2;
  double w0r = 0, w0i = 0, w1r = 0, w1i = 0;
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
    for (int e = tid; e < 64 * 32; e += 256) {
      const int rr = e % 64, c = e / 64, i = r0 + rr;
      cx<T> v = {0, 0};
      if (i < n && c < ncols) v = C[(size_t)(cbeg + c) * P.ldc + i];
      Cs[rr][c] = v;
    }
    __syncthreads();
    const int rmax = min(64, n - r0);
    for (int rr = 0; rr < rmax; ++rr) {
      const cx<T> v = Vs[rr][wa];
      const cx<T> x0 = Cs[rr][wc], x1 = Cs[rr][wc + 1];
      const double vr = v.re, vi = v.im;
      w0r += vr * x0.re + vi * x0.im;
      w0i += vr * x0.im - vi * x0.re;
      w1r += vr * x1.re + vi * x1.im;
      w1i += vr * x1.im - vi * x1.re;
    }
    __syncthreads();
  }
  W1[wa][wc] = cx<double>{w0r, w0i};
  W1[wa][wc + 1] = cx<double>{w1r, w1i};
  __syncthreads();
  // W2 = op(T) W1, kept in registers of the thread that owns (wa, wc..wc+1)
  double y0r = 0, y0i = 0, y1r = 0, y1i = 0;
  for (int b = 0; b < QNB; ++b) {
    const cx<double> t = Tl[wa][b], u0 = W1[b][wc], u1 = W1[b][wc + 1];
    y0r += t.re * u0.re - t.im * u0.im;
    y0i += t.re * u0.im + t.im * u0.re;
    y1r += t.re * u1.re - t.im * u1.im;
    y1i += t.re * u1.im + t.im * u1.re;
  }
  __syncthreads();
  W1[wa][wc] = cx<double>{y0r, y0i};
  W1[wa][wc + 1] = cx<double>{y1r, y1i};
  __syncthreads();
  // C -= V W2
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
    __syncthreads();
    for (int e = tid; e < 64 * 32; e += 256) {
      const int rr = e % 64, c = e / 64, i = r0 + rr;
      if (i < n && c < ncols) {
        double sr = 0, si = 0;
#pragma unroll
        for (int a = 0; a < QNB; ++a) {
          const cx<T> v = Vs[rr][a];
          const cx<double> w = W1[a][c];
          sr += (double)v.re * w.re - (double)v.im * w.im;
          si += (double)v.re * w.im + (double)v.im * w.re;
        }
        cx<T>* p = C + (size_t)(cbeg + c) * P.ldc + i;
        const cx<T> x = *p;
        *p = cx<T>{(T)((double)x.re - sr), (T)((double)x.im - si)};
      }
    }
    __syncthreads();
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
  const int gx = (maxcols + 31) / 32;
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

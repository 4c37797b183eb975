// HIP kernels of libmpo for gfx950 (CDNA4).
//
//   k_gemm         complex GEMM on real MFMA (4M: four real products per
//                  complex K step), LDS-staged 64x64 tiles, batched
//   k_gate         gate pair (G_out (x) G_in^T) on the physical legs of theta,
//                  lambda scaling, (lambda theta)^dag for the QR preconditioner
//   k_jac_init / k_jac_sweep_end   state of the block Jacobi SVD (steps: jacobi.hip)
//   k_colnorms     singular values as column norms (FP64)
//   k_unit_cols    the converged columns scaled to unit length
//   k_col_order / k_permute_cols   columns by decreasing norm (second-QR route)
//   k_sort_trunc   descending sort + truncation decision (FP64)
//   k_env / k_greedy  peak readout of M|0...0> (FP64)
//   k_sample_pick  one site of conditional sampling of M|0...0> for many samples (FP64)
#include "common.h"

namespace mpo {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
template <typename T> struct V4;
template <> struct V4<float> { typedef v4f t; };
template <> struct V4<double> { typedef v4d t; };

__device__ __forceinline__ v4f mfma16x16x4(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4d mfma16x16x4(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ============================================================== GEMM
// One 256-thread workgroup computes a 64x64 complex tile; wave w owns the
// 32x32 quadrant (w>>1, w&1) as 2x2 MFMA 16x16 tiles.  A 16x16x4 MFMA takes
// A[i][k] from lane i + 16k and B[k][j] from lane j + 16k.  Element r of the
// result holds D[4*(lane>>4) + r][lane & 15] for the f32 instruction and
// D[(lane>>4) + 4*r][lane & 15] for the f64 one (measured on gfx950).
constexpr int GT = GEMM_TILE;
constexpr int GK = 16;

template <typename T> __device__ __forceinline__ int mfma_row(int lane, int r);
template <> __device__ __forceinline__ int mfma_row<float>(int lane, int r) { return 4 * (lane >> 4) + r; }
template <> __device__ __forceinline__ int mfma_row<double>(int lane, int r) { return (lane >> 4) + 4 * r; }

template <typename T>
__global__ __launch_bounds__(256) void k_gemm(GemmBatch gb) {
  const int pi = blockIdx.z;
  if (pi >= gb.count) return;
  const GemmProb P = gb.p[pi];
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  if (m0 >= P.M || n0 >= P.N) return;
  if (P.herm && m0 >= n0 + GT) return;
  __shared__ cx<T> As[GT][GK + 1];
  __shared__ cx<T> Bs[GK][GT + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  typedef typename V4<T>::t acc_t;
  acc_t accr[2][2], acci[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 4; ++r) { accr[i][j][r] = 0; acci[i][j][r] = 0; }
  const cx<T>* A = (const cx<T>*)P.A;
  const cx<T>* B = (const cx<T>*)P.B;
  // The next K-slab of both tiles is loaded into registers while the current
  // one is multiplied.  Every load goes to a clamped valid address; the value
  // is masked (multiplied by 0 or 1) only when it is written to LDS, so a
  // thread's loads stay in flight together instead of each being waited for
  // behind a bounds branch.  B's two layouts share one address formula.
  cx<T> an[4], bn[4];
  const bool bt = P.bmode != 0;                                  // B given as op(W) = conj(W)^T
  const int ar = tid >> 2, akk = (tid & 3) * 4;                  // A: row, first k
  const int br0 = bt ? (tid >> 2) : (tid >> 4);                  // B: k row (or n row)
  const int bc0 = bt ? (tid & 3) * 4 : (tid & 15) * 4;           // B: first n (or k)
  const int browmax = bt ? P.N - 1 : P.K - 1, bcolmax = bt ? P.K - 1 : P.N - 1;
  const T bsign = bt ? (T)-1 : (T)1;
  auto load = [&](int k0) {
    const cx<T>* arow = A + (size_t)min(m0 + ar, P.M - 1) * P.lda;
#pragma unroll
    for (int u = 0; u < 4; ++u) an[u] = arow[min(k0 + akk + u, P.K - 1)];
    const int brow = (bt ? n0 : k0) + br0, bcol = (bt ? k0 : n0) + bc0;
    const cx<T>* bp = B + (size_t)min(brow, browmax) * P.ldb;
#pragma unroll
    for (int u = 0; u < 4; ++u) bn[u] = bp[min(bcol + u, bcolmax)];
  };
  load(0);
  for (int k0 = 0; k0 < P.K; k0 += GK) {
    {
      const bool arow_ok = m0 + ar < P.M;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const T mk = (arow_ok && k0 + akk + u < P.K) ? (T)1 : (T)0;
        As[ar][akk + u] = cx<T>{mk * an[u].re, mk * an[u].im};
      }
      const int brow = (bt ? n0 : k0) + br0, bcol = (bt ? k0 : n0) + bc0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const T mk = (brow <= browmax && bcol + u <= bcolmax) ? (T)1 : (T)0;
        const cx<T> v{mk * bn[u].re, bsign * mk * bn[u].im};
        if (bt) Bs[bc0 + u][br0] = v;
        else Bs[br0][bc0 + u] = v;
      }
    }
    __syncthreads();
    if (k0 + GK < P.K) load(k0 + GK);
#pragma unroll
    for (int kk = 0; kk < GK; kk += 4) {
      cx<T> a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = As[wm + t * 16 + (lane & 15)][kk + (lane >> 4)];
        b[t] = Bs[kk + (lane >> 4)][wn + t * 16 + (lane & 15)];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          accr[i][j] = mfma16x16x4(a[i].re, b[j].re, accr[i][j]);
          accr[i][j] = mfma16x16x4(-a[i].im, b[j].im, accr[i][j]);
          acci[i][j] = mfma16x16x4(a[i].re, b[j].im, acci[i][j]);
          acci[i][j] = mfma16x16x4(a[i].im, b[j].re, acci[i][j]);
        }
    }
    __syncthreads();
  }
  cx<T>* C = (cx<T>*)P.C;
  const cx<T>* C0 = (const cx<T>*)P.C0;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + i * 16 + mfma_row<T>(lane, r);
        const int col = n0 + wn + j * 16 + (lane & 15);
        if (row < P.M && col < P.N) {
          cx<T> v{accr[i][j][r], acci[i][j][r]};
          if (C0) {
            const cx<T> c0 = C0[(size_t)row * P.ldc + col];
            v.re += c0.re;
            v.im += c0.im;
          }
          C[(size_t)row * P.ldc + col] = v;
        }
      }
}

// ============================================================== gate
// T[(s1' s2'), (s1 s2)] = G_out[(o1' o2'), (o1 o2)] * G_in[(p1 p2), (p1' p2')],
// s = 2o + p.  One thread per (a, b) applies T to the 16 entries theta0[a, :, :, b].
template <typename T>
__global__ __launch_bounds__(256) void k_gate(GateBatch gb) {
  const int pi = blockIdx.y;
  if (pi >= gb.count) return;
  const GateProb P = gb.p[pi];
  __shared__ cx<T> Tm[16][16];
  const int tid = threadIdx.x;
  {
    const int row = tid >> 4, col = tid & 15;
    const int s1p = row >> 2, s2p = row & 3, s1 = col >> 2, s2 = col & 3;
    const int o1p = s1p >> 1, p1p = s1p & 1, o2p = s2p >> 1, p2p = s2p & 1;
    const int o1 = s1 >> 1, p1 = s1 & 1, o2 = s2 >> 1, p2 = s2 & 1;
    double gre, gim, hre, him;
    if (P.has_out) {
      const int idx = ((o1p * 2 + o2p) * 4 + (o1 * 2 + o2)) * 2;
      gre = P.gates[idx];
      gim = P.gates[idx + 1];
    } else {
      gre = (o1p == o1 && o2p == o2) ? 1.0 : 0.0;
      gim = 0.0;
    }
    if (P.has_in) {
      const int idx = 32 + ((p1 * 2 + p2) * 4 + (p1p * 2 + p2p)) * 2;
      hre = P.gates[idx];
      him = P.gates[idx + 1];
    } else {
      hre = (p1 == p1p && p2 == p2p) ? 1.0 : 0.0;
      him = 0.0;
    }
    Tm[row][col] = cx<T>{(T)(gre * hre - gim * him), (T)(gre * him + gim * hre)};
  }
  __syncthreads();
  const int chir = P.chir, n = 4 * chir;
  const int total = P.chil * chir;
  const cx<T>* th0 = (const cx<T>*)P.theta0;
  cx<T>* thn = (cx<T>*)P.theta_nolam;
  cx<T>* Mo = (cx<T>*)P.M;
  for (int idx = blockIdx.x * 256 + tid; idx < total; idx += gridDim.x * 256) {
    const int a = idx / chir, b = idx - a * chir;
    cx<T> in[16];
#pragma unroll
    for (int s1 = 0; s1 < 4; ++s1)
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) in[s1 * 4 + s2] = th0[(size_t)(4 * a + s1) * n + s2 * chir + b];
    const T lam = (T)P.lam[a];
    // every input of this thread is read before any output is written, so
    // M may alias theta0
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      T re = 0, im = 0;
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        const cx<T> t = Tm[r][c];
        re += t.re * in[c].re - t.im * in[c].im;
        im += t.re * in[c].im + t.im * in[c].re;
      }
      const int s1p = r >> 2, s2p = r & 3;
      thn[(size_t)(4 * a + s1p) * n + s2p * chir + b] = cx<T>{re, im};
      Mo[(size_t)(4 * a + s1p) * n + s2p * chir + b] = cx<T>{re * lam, -im * lam};
    }
  }
}

// ============================================================== Jacobi SVD
// Round-robin (circle method) pairing of N items (N even): over N-1 steps
// every pair meets exactly once; step s pairs (s, N-1) and (s+t, s-t) mod N-1.
__device__ __forceinline__ void rr_pair(int N, int step, int t, int& a, int& b) {
  if (t == 0) {
    a = step;
    b = N - 1;
  } else {
    a = (step + t) % (N - 1);
    b = (step - t + (N - 1)) % (N - 1);
  }
  if (a > b) {
    const int x = a;
    a = b;
    b = x;
  }
}

template <typename T>
__global__ void k_jac_init(JacBatch jb) {
  const int pi = blockIdx.y;
  if (pi >= jb.count) return;
  const JacProb P = jb.p[pi];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    P.st->active = 1;
    P.st->rot = 0;
    P.st->sweeps = 0;
    P.st->rot_total = 0;
    P.st->epoch = 0;
  }
  // pair-skip bookkeeping starts empty
  const size_t nb = (size_t)P.nblk;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nb * nb + nb;
       i += (size_t)gridDim.x * blockDim.x) {
    if (i < nb * nb) P.pchk[i] = 0;
    else P.bmod[i - nb * nb] = 0;
  }
  const size_t npad = (size_t)P.ncol_pad;
  const size_t nv = P.V ? npad * npad : 0;
  const size_t na = (size_t)(P.ncol_pad - P.ncol) * P.lda;
  cx<T>* V = (cx<T>*)P.V;
  cx<T>* A = (cx<T>*)P.A + (size_t)P.ncol * P.lda;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv + na; i += (size_t)gridDim.x * blockDim.x) {
    if (i < nv) {
      const size_t r = i % npad, c = i / npad;
      V[i] = cx<T>{(T)(r == c ? 1 : 0), (T)0};
    } else {
      A[i - nv] = cx<T>{0, 0};
    }
  }
}

__global__ void k_jac_sweep_end(JacBatch jb) {
  const int i = threadIdx.x;
  if (i >= jb.count) return;
  JacState* s = jb.p[i].st;
  s->epoch += 1;
  if (s->active) {
    s->sweeps += 1;
    s->rot_total += s->rot;
    if (s->rot == 0) s->active = 0;
    s->rot = 0;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_colnorms(JacBatch jb) {
  const int pi = blockIdx.y;
  if (pi >= jb.count) return;
  const JacProb P = jb.p[pi];
  const int lane = threadIdx.x & 63;
  const int col = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (col >= P.ncol_pad) return;
  const cx<T>* A = (const cx<T>*)P.A + (size_t)col * P.lda;
  double acc = 0.0;
  if (col < P.ncol)
    for (int r = lane; r < P.m; r += 64) {
      const double xr = A[r].re, xi = A[r].im;
      acc += xr * xr + xi * xi;
    }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) P.norms[col] = sqrt(acc);
}

// U = A diag(1 / norms): the converged operand's columns scaled to unit
// length (their directions are the singular vectors the second-QR route
// keeps), into V (column-major, ncol_pad x ncol_pad); rows past m, columns
// past ncol and columns of zero norm are zero.  One workgroup per column.
template <typename T>
__global__ __launch_bounds__(256) void k_unit_cols(JacBatch jb) {
  const int pi = blockIdx.y;
  if (pi >= jb.count) return;
  const JacProb P = jb.p[pi];
  const int col = blockIdx.x;
  if (col >= P.ncol_pad) return;
  const double nrm = col < P.ncol ? P.norms[col] : 0.0;
  const T sc = nrm > 0.0 ? (T)(1.0 / nrm) : (T)0;
  const cx<T>* A = (const cx<T>*)P.A + (size_t)min(col, P.ncol_pad - 1) * P.lda;
  cx<T>* U = (cx<T>*)P.V + (size_t)col * P.ncol_pad;
  for (int r = threadIdx.x; r < P.ncol_pad; r += 256) {
    const cx<T> x = A[min(r, P.m - 1)];
    const T mk = r < P.m ? sc : (T)0;
    U[r] = cx<T>{mk * x.re, mk * x.im};
  }
}

// Columns by decreasing norm (ties by index; a non-finite norm sorts first,
// so it stays among the real columns and the truncation still reports it;
// padding columns last), and the pair-skip bookkeeping cleared.  One
// workgroup per problem, bitonic sort in LDS.
__global__ __launch_bounds__(1024) void k_col_order(ColSortBatch cb) {
  const int pi = blockIdx.x;
  if (pi >= cb.count) return;
  const ColSortProb P = cb.p[pi];
  if (!P.on) return;
  __shared__ double key[4096];
  __shared__ int idx[4096];
  int N2 = 1;
  while (N2 < P.ncol_pad) N2 <<= 1;
  for (int i = threadIdx.x; i < N2; i += blockDim.x) {
    double v = (i < P.ncol) ? P.norms[i] : -1.0;
    if (!isfinite(v)) v = __builtin_huge_val();
    key[i] = (i < P.ncol_pad) ? v : -2.0;
    idx[i] = i;
  }
  const int nb = P.nblk;
  for (int i = threadIdx.x; i < nb * nb + nb; i += blockDim.x) {
    if (i < nb * nb) P.pchk[i] = 0;
    else P.bmod[i - nb * nb] = 0;
  }
  __syncthreads();
  for (int k = 2; k <= N2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < N2; i += blockDim.x) {
        const int l = i ^ j;
        if (l > i) {
          const bool up = ((i & k) == 0);
          const double ki = key[i], kl = key[l];
          const int ii = idx[i], il = idx[l];
          const bool l_before_i = (kl > ki) || (kl == ki && il < ii);
          if (up ? l_before_i : !l_before_i) {
            key[i] = kl;
            key[l] = ki;
            idx[i] = il;
            idx[l] = ii;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < P.ncol_pad; i += blockDim.x) P.perm[i] = idx[i];
}

// A2[:, j] = A[:, perm[j]] over the m used rows: column blockIdx.x, rows in
// chunks of 1024 (blockIdx.y).
template <typename T>
__global__ __launch_bounds__(256) void k_permute_cols(ColSortBatch cb) {
  const int pi = blockIdx.z;
  if (pi >= cb.count) return;
  const ColSortProb P = cb.p[pi];
  if (!P.on) return;
  const int j = blockIdx.x;
  if (j >= P.ncol_pad) return;
  const int r0 = blockIdx.y * 1024;
  if (r0 >= P.m) return;
  const cx<T>* src = (const cx<T>*)P.A + (size_t)P.perm[j] * P.lda;
  cx<T>* dst = (cx<T>*)P.A2 + (size_t)j * P.lda;
  const int r1 = min(P.m, r0 + 1024);
  for (int r = r0 + threadIdx.x; r < r1; r += 256) dst[r] = src[r];
}

// ============================================================== sort + truncation
__global__ __launch_bounds__(1024) void k_sort_trunc(TruncBatch tb) {
  const int pi = blockIdx.x;
  if (pi >= tb.count) return;
  const TruncProb P = tb.p[pi];
  __shared__ double key[4096];
  __shared__ int idx[4096];
  __shared__ int nonfinite;
  int N2 = 1;
  while (N2 < P.ncol_pad) N2 <<= 1;
  if (threadIdx.x == 0) nonfinite = 0;
  __syncthreads();
  // A non-finite norm is flagged before anything else reads it and enters the
  // sort as -1 (every comparison with NaN is false, which would break the
  // sorting network), so the result is an error, never a silent zero.
  for (int i = threadIdx.x; i < N2; i += blockDim.x) {
    double v = (i < P.ncol) ? P.norms[i] : -1.0;
    if (!isfinite(v)) {
      nonfinite = 1;
      v = -1.0;
    }
    key[i] = v;
    idx[i] = i;
  }
  __syncthreads();
  // bitonic sort: descending key, ascending index on ties
  for (int k = 2; k <= N2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < N2; i += blockDim.x) {
        const int l = i ^ j;
        if (l > i) {
          const bool up = ((i & k) == 0);
          const double ki = key[i], kl = key[l];
          const int ii = idx[i], il = idx[l];
          // "before(x, y)": x sorts ahead of y
          const bool l_before_i = (kl > ki) || (kl == ki && il < ii);
          if (up ? l_before_i : !l_before_i) {
            key[i] = kl;
            key[l] = ki;
            idx[i] = il;
            idx[l] = ii;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < P.ncol; i += blockDim.x) {
    P.s_sorted[i] = key[i] > 0.0 ? key[i] : 0.0;
    P.perm[i] = idx[i];
  }
  if (threadIdx.x == 0) {
    const int nvals = P.nval;
    int bad = 0;
    double total = 0.0;
    for (int j = nvals - 1; j >= 0; --j) {
      const double s = key[j] > 0.0 ? key[j] : 0.0;
      if (!isfinite(s)) bad = 1;
      total += s * s;
    }
    const double s0 = key[0] > 0.0 ? key[0] : 0.0;
    int k;
    if (P.mode == 0) {
      k = 0;
      for (int j = 0; j < nvals; ++j)
        if (key[j] > P.cutoff * s0) ++k;
    } else {
      const double thr = P.cutoff * total;
      double tail = 0.0;
      k = 0;
      for (int j = nvals - 1; j >= 0; --j) {
        const double s = key[j] > 0.0 ? key[j] : 0.0;
        tail += s * s;
        if (tail > thr) {
          k = j + 1;
          break;
        }
      }
    }
    if (k > P.chi_max) k = P.chi_max;
    if (k > nvals) k = nvals;
    if (k < 1) k = 1;
    double disc = 0.0;
    for (int j = nvals - 1; j >= k; --j) {
      const double s = key[j] > 0.0 ? key[j] : 0.0;
      disc += s * s;
    }
    P.res->k = k;
    P.res->nvals = nvals;
    P.res->discarded = disc;
    P.res->total = total;
    P.res->s0 = s0;
    P.res->bad = bad || nonfinite || !isfinite(total);
  }
}

// ============================================================== peak readout
// C[i][j] (+)= sum_k opA(i,k) opB(k,j); opX(i,k) = X[off + i*s0 + k*s1] (conj if cX)
template <typename TA, typename TB>
__global__ __launch_bounds__(256) void k_zgemm_small(cx<double>* C, int ldc, const cx<TA>* A, long long as0,
                                                      long long as1, int cA, const cx<TB>* B, long long bs0,
                                                      long long bs1, int cB, int M, int N, int K, int beta) {
  __shared__ cx<double> As[16][17], Bs[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i = blockIdx.y * 16 + ty, j = blockIdx.x * 16 + tx;
  double cr = 0, ci = 0;
  for (int k0 = 0; k0 < K; k0 += 16) {
    {
      const int ii = blockIdx.y * 16 + ty, kk = k0 + tx;
      cx<double> v = {0, 0};
      if (ii < M && kk < K) {
        const cx<TA> x = A[ii * as0 + kk * as1];
        v = cx<double>{(double)x.re, cA ? -(double)x.im : (double)x.im};
      }
      As[ty][tx] = v;
    }
    {
      const int kk = k0 + ty, jj = blockIdx.x * 16 + tx;
      cx<double> v = {0, 0};
      if (kk < K && jj < N) {
        const cx<TB> x = B[kk * bs0 + jj * bs1];
        v = cx<double>{(double)x.re, cB ? -(double)x.im : (double)x.im};
      }
      Bs[ty][tx] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const cx<double> a = As[ty][k], b = Bs[k][tx];
      cr += a.re * b.re - a.im * b.im;
      ci += a.re * b.im + a.im * b.re;
    }
    __syncthreads();
  }
  if (i < M && j < N) {
    cx<double>* c = C + (size_t)i * ldc + j;
    if (beta) {
      c->re += cr;
      c->im += ci;
    } else {
      *c = cx<double>{cr, ci};
    }
  }
}

// One workgroup: w_o = v A_o (o = 0, 1), p_o = w_o E w_o^dag, pick the larger
// (ties -> 0), v <- w_o / |w_o|, accumulate log of the conditional.
template <typename T>
__global__ __launch_bounds__(1024) void k_greedy(const cx<T>* site, int chil, int chir, const cx<double>* E,
                                                 const cx<double>* v, cx<double>* vout, cx<double>* work,
                                                 unsigned char* bit_out, double* logp) {
  __shared__ double red[2][1024];
  __shared__ int choice;
  __shared__ double nrm;
  const int tid = threadIdx.x;
  cx<double>* w0 = work;
  cx<double>* w1 = work + chir;
  for (int b = tid; b < chir; b += blockDim.x) {
    double r0 = 0, i0 = 0, r1 = 0, i1 = 0;
    for (int a = 0; a < chil; ++a) {
      const cx<double> va = v[a];
      const cx<T> x0 = site[(size_t)a * 4 * chir + 0 * chir + b];
      const cx<T> x1 = site[(size_t)a * 4 * chir + 2 * chir + b];
      r0 += va.re * (double)x0.re - va.im * (double)x0.im;
      i0 += va.re * (double)x0.im + va.im * (double)x0.re;
      r1 += va.re * (double)x1.re - va.im * (double)x1.im;
      i1 += va.re * (double)x1.im + va.im * (double)x1.re;
    }
    w0[b] = cx<double>{r0, i0};
    w1[b] = cx<double>{r1, i1};
  }
  __syncthreads();
  double p0 = 0, p1 = 0;
  for (int b = tid; b < chir; b += blockDim.x) {
    // y_o[b] = sum_b' E[b][b'] conj(w_o[b']);  p_o += w_o[b] y_o[b]
    double y0r = 0, y0i = 0, y1r = 0, y1i = 0;
    for (int bp = 0; bp < chir; ++bp) {
      const cx<double> e = E[(size_t)b * chir + bp];
      const cx<double> a0 = w0[bp], a1 = w1[bp];
      y0r += e.re * a0.re + e.im * a0.im;
      y0i += e.im * a0.re - e.re * a0.im;
      y1r += e.re * a1.re + e.im * a1.im;
      y1i += e.im * a1.re - e.re * a1.im;
    }
    p0 += w0[b].re * y0r - w0[b].im * y0i;
    p1 += w1[b].re * y1r - w1[b].im * y1i;
  }
  red[0][tid] = p0;
  red[1][tid] = p1;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) {
      red[0][tid] += red[0][tid + s];
      red[1][tid] += red[1][tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double q0 = red[0][0], q1 = red[1][0];
    const int o = (q1 > q0) ? 1 : 0;
    choice = o;
    *bit_out = (unsigned char)o;
    *logp += log((o ? q1 : q0) / (q0 + q1));
  }
  __syncthreads();
  const cx<double>* w = choice ? w1 : w0;
  double ss = 0;
  for (int b = tid; b < chir; b += blockDim.x) ss += w[b].re * w[b].re + w[b].im * w[b].im;
  red[0][tid] = ss;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) red[0][tid] += red[0][tid + s];
    __syncthreads();
  }
  if (tid == 0) nrm = sqrt(red[0][0]);
  __syncthreads();
  const double inv = nrm > 0 ? 1.0 / nrm : 0.0;
  for (int b = tid; b < chir; b += blockDim.x) vout[b] = cx<double>{w[b].re * inv, w[b].im * inv};
}

// Sampling (one workgroup per sample s): with X_o = L A_o and Y_o = X_o E
// (row s of each, cr entries), p_o = Re sum_c Y_o[c] conj(X_o[c]); the bit is
// 0 when u < p_0 / (p_0 + p_1); the log of the chosen conditional is added to
// logp[s] and the next left vector is X_o / sqrt(p_o).  The sums run in a
// fixed order (strided per thread, then a tree), so a sample's decisions do
// not depend on the launch.  A non-finite or non-positive p_0 + p_1 sets
// *bad.
__global__ __launch_bounds__(256) void k_sample_pick(const cx<double>* X, const cx<double>* Y, int count, int cr,
                                                     const double* u, int ustride, cx<double>* Lout, double* logp,
                                                     unsigned char* bits, int bstride, int* bad) {
  __shared__ double red[2][256];
  __shared__ int choice;
  __shared__ double scale;
  const int s = blockIdx.x, tid = threadIdx.x;
  if (s >= count) return;
  const size_t plane = (size_t)count * cr;
  const cx<double>* x0 = X + (size_t)s * cr;
  const cx<double>* y0 = Y + (size_t)s * cr;
  double p0 = 0, p1 = 0;
  for (int c = tid; c < cr; c += 256) {
    const cx<double> a0 = x0[c], b0 = y0[c], a1 = x0[plane + c], b1 = y0[plane + c];
    p0 += b0.re * a0.re + b0.im * a0.im;
    p1 += b1.re * a1.re + b1.im * a1.im;
  }
  red[0][tid] = p0;
  red[1][tid] = p1;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      red[0][tid] += red[0][tid + w];
      red[1][tid] += red[1][tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double q0 = red[0][0], q1 = red[1][0], tot = q0 + q1;
    int o = 0;
    if (!(tot > 0) || !isfinite(tot) || q0 < 0 || q1 < 0) {
      *bad = 1;
      scale = 0;
    } else {
      o = (u[(size_t)s * ustride] < q0 / tot) ? 0 : 1;
      const double q = o ? q1 : q0;
      logp[s] += log(q / tot);
      scale = q > 0 ? 1.0 / sqrt(q) : 0.0;
    }
    choice = o;
    bits[(size_t)s * bstride] = (unsigned char)o;
  }
  __syncthreads();
  const cx<double>* xs = x0 + (choice ? plane : 0);
  const double f = scale;
  for (int c = tid; c < cr; c += 256) Lout[(size_t)s * cr + c] = cx<double>{xs[c].re * f, xs[c].im * f};
}

template <typename TD, typename TS>
__global__ void k_convert(cx<TD>* dst, const cx<TS>* src, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = cx<TD>{(TD)src[i].re, (TD)src[i].im};
}

// ============================================================== launchers
template <typename T>
void launch_gemm(const GemmBatch& b, int maxM, int maxN, hipStream_t s) {
  dim3 grid((maxN + GT - 1) / GT, (maxM + GT - 1) / GT, b.count);
  hipLaunchKernelGGL(k_gemm<T>, grid, dim3(256), 0, s, b);
}
template <typename T>
void launch_gate(const GateBatch& b, int maxtotal, hipStream_t s) {
  int gx = (maxtotal + 255) / 256;
  if (gx > 512) gx = 512;
  if (gx < 1) gx = 1;
  hipLaunchKernelGGL(k_gate<T>, dim3(gx, b.count), dim3(256), 0, s, b);
}
template <typename T>
void launch_jac_init(const JacBatch& b, hipStream_t s) {
  hipLaunchKernelGGL(k_jac_init<T>, dim3(256, b.count), dim3(256), 0, s, b);
}
void launch_jac_sweep_end(const JacBatch& b, hipStream_t s) {
  hipLaunchKernelGGL(k_jac_sweep_end, dim3(1), dim3(64), 0, s, b);
}
template <typename T>
void launch_colnorms(const JacBatch& b, int maxcols, hipStream_t s) {
  hipLaunchKernelGGL(k_colnorms<T>, dim3((maxcols + 3) / 4, b.count), dim3(256), 0, s, b);
}
template <typename T>
void launch_col_order(const ColSortBatch& b, int maxcols, int maxrows, hipStream_t s) {
  hipLaunchKernelGGL(k_col_order, dim3(b.count), dim3(1024), 0, s, b);
  hipLaunchKernelGGL(k_permute_cols<T>, dim3(maxcols, (maxrows + 1023) / 1024, b.count), dim3(256), 0, s, b);
}
template <typename T>
void launch_unit_cols(const JacBatch& b, int maxcols, hipStream_t s) {
  hipLaunchKernelGGL(k_unit_cols<T>, dim3(maxcols, b.count), dim3(256), 0, s, b);
}
void launch_sort_trunc(const TruncBatch& b, hipStream_t s) {
  hipLaunchKernelGGL(k_sort_trunc, dim3(b.count), dim3(1024), 0, s, b);
}
template <typename TA, typename TB>
void launch_zgemm_small(cx<double>* C, int ldc, const cx<TA>* A, long long as0, long long as1, int cA,
                        const cx<TB>* B, long long bs0, long long bs1, int cB, int M, int N, int K, int beta,
                        hipStream_t s) {
  dim3 grid((N + 15) / 16, (M + 15) / 16);
  hipLaunchKernelGGL((k_zgemm_small<TA, TB>), grid, dim3(256), 0, s, C, ldc, A, as0, as1, cA, B, bs0, bs1, cB, M,
                     N, K, beta);
}
template <typename T>
void launch_greedy(const cx<T>* site, int chil, int chir, const cx<double>* E, const cx<double>* v,
                   cx<double>* vout, cx<double>* work, unsigned char* bit, double* logp, hipStream_t s) {
  hipLaunchKernelGGL(k_greedy<T>, dim3(1), dim3(1024), 0, s, site, chil, chir, E, v, vout, work, bit, logp);
}
void launch_sample_pick(const cx<double>* X, const cx<double>* Y, int count, int cr, const double* u, int ustride,
                        cx<double>* Lout, double* logp, unsigned char* bits, int bstride, int* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_sample_pick, dim3(count), dim3(256), 0, s, X, Y, count, cr, u, ustride, Lout, logp, bits,
                     bstride, bad);
}
template <typename TD, typename TS>
void launch_convert(cx<TD>* d, const cx<TS>* src, size_t n, hipStream_t s) {
  size_t g = (n + 255) / 256;
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  hipLaunchKernelGGL((k_convert<TD, TS>), dim3((unsigned)g), dim3(256), 0, s, d, src, n);
}

#define INST(T)                                                                                          \
  template void launch_gemm<T>(const GemmBatch&, int, int, hipStream_t);                                 \
  template void launch_gate<T>(const GateBatch&, int, hipStream_t);                                      \
  template void launch_jac_init<T>(const JacBatch&, hipStream_t);                                        \
  template void launch_colnorms<T>(const JacBatch&, int, hipStream_t);                                   \
  template void launch_unit_cols<T>(const JacBatch&, int, hipStream_t);                                  \
  template void launch_col_order<T>(const ColSortBatch&, int, int, hipStream_t);                         \
  template void launch_greedy<T>(const cx<T>*, int, int, const cx<double>*, const cx<double>*,           \
                                 cx<double>*, cx<double>*, unsigned char*, double*, hipStream_t);

INST(float)
INST(double)

#define INST2(TA, TB)                                                                                    \
  template void launch_zgemm_small<TA, TB>(cx<double>*, int, const cx<TA>*, long long, long long, int,   \
                                           const cx<TB>*, long long, long long, int, int, int, int, int, \
                                           hipStream_t);                                                 \
  template void launch_convert<TA, TB>(cx<TA>*, const cx<TB>*, size_t, hipStream_t);

INST2(float, double)
INST2(double, float)
INST2(double, double)

}  // namespace mpo

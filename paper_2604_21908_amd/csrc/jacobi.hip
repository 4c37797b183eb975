// Block one-sided Jacobi SVD steps (gfx950).
//
// Columns of the operand are grouped in blocks of JB = 16; a round-robin step
// pairs every block with one other, giving 32-column panels P that are
// processed independently:
//
//   k_jac_gram  partial Gram matrices P^dag P over row chunks of GRC rows on
//               MFMA (f32 16x16x4 with an FP64 sum per 64-row slab, or f64);
//               grid = pairs x row chunks x problems
//   k_jac_evd   per panel: FP64 sum of the partial Grams, convergence test,
//               at most one or two sweeps of cyclic Jacobi on G with FP64
//               angles (the outer iteration finishes what they leave), and
//               D = W - I rounded to the working precision
//   k_jac_rot   P <- P + P D on MFMA over row chunks of RRC rows of theta's
//               and V's panels, computed as P^T <- P^T + D^T P^T so that
//               each 16-lane group of a wave reads and writes 16 consecutive
//               rows of one column
//   k_jac_gram_bf16 / k_jac_rot_mixed  the mixed form: Gram matrices with
//               split-BF16 products, and one rotation launch in which theta's
//               row chunks use split-BF16 products while the accumulated
//               rotations V stay on FP32 MFMA (the EVD stays FP64)
#include "common.h"
#include "mfma.h"

namespace mpo {

// Inner cyclic-Jacobi sweeps per panel EVD (a kernel argument): two already
// give the outer iteration its full convergence rate, more only add latency;
// one costs about one extra outer sweep but halves the EVD.

__device__ __forceinline__ void rr_pair2(int N, int step, int t, int& a, int& b) {
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

__device__ __forceinline__ int panel_col(int bi, int bj, int c) { return c < JB ? bi * JB + c : bj * JB + c - JB; }

// ---------------------------------------------------------------- Gram
template <typename T>
__global__ __launch_bounds__(256) void k_jac_gram(JacBatch jb, int step) {
  const int pi = blockIdx.z;
  if (pi >= jb.count) return;
  const JacProb P = jb.p[pi];
  if (step >= P.nblk - 1 || (int)blockIdx.x >= P.nblk / 2) return;
  if (P.st->active == 0) return;
  const int r0 = blockIdx.y * GRC;
  if (r0 >= P.m) return;
  const int r1 = min(P.m, r0 + GRC);
  int bi, bj;
  rr_pair2(P.nblk, step, blockIdx.x, bi, bj);
  if (pair_unchanged(P, bi, bj)) return;
  __shared__ cx<T> Pc[64][33];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int I = wave >> 1, J = wave & 1;
  const cx<T>* A = (const cx<T>*)P.A;
  typedef typename MF<T>::acc acc_t;
  double gr[4] = {0, 0, 0, 0}, gi[4] = {0, 0, 0, 0};
  // the next 64-row slab is loaded into registers while this one is multiplied
  cx<T> nxt[8];
  auto fetch = [&](int s0) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int c = wave + 4 * u;
      nxt[u] = cx<T>{0, 0};
      if (s0 + lane < r1) nxt[u] = A[(size_t)panel_col(bi, bj, c) * P.lda + s0 + lane];
    }
  };
  fetch(r0);
  for (int s0 = r0; s0 < r1; s0 += 64) {
#pragma unroll
    for (int u = 0; u < 8; ++u) Pc[lane][wave + 4 * u] = nxt[u];
    __syncthreads();
    if (s0 + 64 < r1) fetch(s0 + 64);
    acc_t are = {0, 0, 0, 0}, aim = {0, 0, 0, 0};
#pragma unroll 4
    for (int kk = 0; kk < 64; kk += 4) {
      const cx<T> x = Pc[kk + (lane >> 4)][I * 16 + (lane & 15)];   // A = P^dag: conj applied below
      const cx<T> y = Pc[kk + (lane >> 4)][J * 16 + (lane & 15)];
      are = MF<T>::mma(x.re, y.re, are);
      are = MF<T>::mma(x.im, y.im, are);
      aim = MF<T>::mma(x.re, y.im, aim);
      aim = MF<T>::mma(-x.im, y.re, aim);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      gr[r] += (double)are[r];
      gi[r] += (double)aim[r];
    }
    __syncthreads();
  }
  cx<double>* out = P.gpart + ((size_t)blockIdx.x * P.ngchunk + blockIdx.y) * 1024;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = I * 16 + MF<T>::row(lane, r), j = J * 16 + (lane & 15);
    out[i * 32 + j] = cx<double>{gr[r], gi[r]};
  }
}

// ---------------------------------------------------------------- EVD
// In a round-robin step the 32 indices form 16 disjoint pairs; the rotation
// J = [[c, z], [-conj(z), c]] of pair k acts on columns (p_k, q_k).  Thread
// (kr, kc) owns the 2x2 block of G at rows (p_kr, q_kr) x columns (p_kc, q_kc)
// and replaces it by J_kr^dag G_block J_kc, and likewise W's rows (p_kr, q_kr)
// x columns (p_kc, q_kc) by W_block J_kc: every entry is read and written by
// exactly one thread, so the update runs in place.
template <typename T>
__global__ __launch_bounds__(256) void k_jac_evd(JacBatch jb, int step, int inner_sweeps, int stamp) {
  const int pi = blockIdx.y;
  if (pi >= jb.count) return;
  const JacProb P = jb.p[pi];
  if (step >= P.nblk - 1 || (int)blockIdx.x >= P.nblk / 2) return;
  if (P.st->active == 0) return;
  const double tol = P.tol;
  __shared__ cx<double> G[32][33];
  __shared__ cx<double> W[32][33];
  __shared__ double rc[16], rzr[16], rzi[16];
  __shared__ int flag, anyrot;
  const int tid = threadIdx.x;
  const int gi = tid >> 3, gj0 = (tid & 7) * 4;
  int* pflag = P.pflag + blockIdx.x;
  int bi, bj;
  rr_pair2(P.nblk, step, blockIdx.x, bi, bj);
  if (pair_unchanged(P, bi, bj)) {
    if (tid == 0) *pflag = 0;
    return;
  }
  // sum of the partial Gram matrices in chunk order (deterministic)
  const int nch = (P.m + GRC - 1) / GRC;
  const cx<double>* gp = P.gpart + (size_t)blockIdx.x * P.ngchunk * 1024;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = gi * 32 + gj0 + u;
    double sr = 0, si = 0;
#pragma unroll 4
    for (int c = 0; c < nch; ++c) {
      const cx<double> v = gp[(size_t)c * 1024 + e];
      sr += v.re;
      si += v.im;
    }
    G[gi][gj0 + u] = cx<double>{sr, si};
    W[gi][gj0 + u] = cx<double>{(gi == gj0 + u) ? 1.0 : 0.0, 0.0};
  }
  if (tid == 0) flag = 0;
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = gj0 + u;
    if (j > gi) {
      const cx<double> g = G[gi][j];
      const double d = G[gi][gi].re * G[j][j].re;
      if (d > 0 && g.re * g.re + g.im * g.im > tol * tol * d) flag = 1;
    }
  }
  __syncthreads();
  if (!flag) {
    if (tid == 0) {
      *pflag = 0;
      P.pchk[bi * P.nblk + bj] = stamp;
    }
    return;
  }
  if (tid == 0) {
    *pflag = 1;
    P.bmod[bi] = stamp;
    P.bmod[bj] = stamp;
    atomicAdd(&P.st->rot, 1);
  }
  const int kr = tid >> 4, kc = tid & 15;
  for (int isw = 0; isw < inner_sweeps; ++isw) {
    if (tid == 0) anyrot = 0;
    __syncthreads();
    for (int st = 0; st < 31; ++st) {
      if (tid < 16) {
        int p, q;
        rr_pair2(32, st, tid, p, q);
        const double app = G[p][p].re, aqq = G[q][q].re;
        const cx<double> g = G[p][q];
        const double mag = sqrt(g.re * g.re + g.im * g.im);
        double c = 1.0, zr = 0.0, zi = 0.0;
        if (mag > 0.0 && mag > tol * sqrt(fmax(app * aqq, 0.0))) {
          const double zeta = (aqq - app) / (2.0 * mag);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          c = 1.0 / sqrt(1.0 + t * t);
          const double s = t * c;
          zr = s * g.re / mag;
          zi = s * g.im / mag;
          anyrot = 1;
        }
        rc[tid] = c;
        rzr[tid] = zr;
        rzi[tid] = zi;
      }
      __syncthreads();
      int pr, qr, pc, qc;
      rr_pair2(32, st, kr, pr, qr);
      rr_pair2(32, st, kc, pc, qc);
      const double cr = rc[kr], zrr = rzr[kr], zri = rzi[kr];
      const double cc = rc[kc], zcr = rzr[kc], zci = rzi[kc];
      if (!(zrr == 0.0 && zri == 0.0 && zcr == 0.0 && zci == 0.0)) {
        // H = G_block J_c, J_c = [[cc, zc], [-conj(zc), cc]]
        const cx<double> a00 = G[pr][pc], a01 = G[pr][qc], a10 = G[qr][pc], a11 = G[qr][qc];
        // x * (-conj(zc)) = -(x.re zcr + x.im zci) + i (x.re zci - x.im zcr)
        const double h00r = a00.re * cc - (a01.re * zcr + a01.im * zci);
        const double h00i = a00.im * cc + (a01.re * zci - a01.im * zcr);
        const double h01r = a00.re * zcr - a00.im * zci + a01.re * cc;
        const double h01i = a00.re * zci + a00.im * zcr + a01.im * cc;
        const double h10r = a10.re * cc - (a11.re * zcr + a11.im * zci);
        const double h10i = a10.im * cc + (a11.re * zci - a11.im * zcr);
        const double h11r = a10.re * zcr - a10.im * zci + a11.re * cc;
        const double h11i = a10.re * zci + a10.im * zcr + a11.im * cc;
        // G' = J_r^dag H, J_r^dag = [[cr, -zr], [conj(zr), cr]]
        G[pr][pc] = cx<double>{cr * h00r - (zrr * h10r - zri * h10i), cr * h00i - (zrr * h10i + zri * h10r)};
        G[pr][qc] = cx<double>{cr * h01r - (zrr * h11r - zri * h11i), cr * h01i - (zrr * h11i + zri * h11r)};
        G[qr][pc] = cx<double>{zrr * h00r + zri * h00i + cr * h10r, zrr * h00i - zri * h00r + cr * h10i};
        G[qr][qc] = cx<double>{zrr * h01r + zri * h01i + cr * h11r, zrr * h01i - zri * h01r + cr * h11i};
      }
      if (!(zcr == 0.0 && zci == 0.0)) {
        // W' = W_block J_c on rows (pr, qr)
        const cx<double> w00 = W[pr][pc], w01 = W[pr][qc], w10 = W[qr][pc], w11 = W[qr][qc];
        W[pr][pc] = cx<double>{w00.re * cc - (w01.re * zcr + w01.im * zci), w00.im * cc + (w01.re * zci - w01.im * zcr)};
        W[pr][qc] = cx<double>{w00.re * zcr - w00.im * zci + w01.re * cc, w00.re * zci + w00.im * zcr + w01.im * cc};
        W[qr][pc] = cx<double>{w10.re * cc - (w11.re * zcr + w11.im * zci), w10.im * cc + (w11.re * zci - w11.im * zcr)};
        W[qr][qc] = cx<double>{w10.re * zcr - w10.im * zci + w11.re * cc, w10.re * zci + w10.im * zcr + w11.im * cc};
      }
      __syncthreads();
    }
    const int any = anyrot;
    __syncthreads();
    if (!any) break;
  }
  // D = W - I, rounded entry by entry (see k_jac_rot)
  cx<T>* D = (cx<T>*)P.dmat + (size_t)blockIdx.x * 1024;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = gi, c = gj0 + u;
    D[r * 32 + c] = cx<T>{(T)(W[r][c].re - (r == c ? 1.0 : 0.0)), (T)W[r][c].im};
  }
}

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
    acc_t cre[2], cim[2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const cx<T> a = Sw[lane & 15][t * 16 + MF<T>::row(lane, r)];
        cre[t][r] = a.re;
        cim[t][r] = a.im;
      }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      const int k = 4 * kk + (lane >> 4);
      const cx<T> x = v[kk];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const cx<T> d = Ds[k][t * 16 + (lane & 15)];   // A[c][k] = D[k][c]
        cre[t] = MF<T>::mma(d.re, x.re, cre[t]);
        cre[t] = MF<T>::mma(-d.im, x.im, cre[t]);
        cim[t] = MF<T>::mma(d.re, x.im, cim[t]);
        cim[t] = MF<T>::mma(d.im, x.re, cim[t]);
      }
    }
    const int rho = s0 + (lane & 15);
    if (rho < c1) {
      const StripBase<T> sb = strip_base<T>(P, rho);
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) sb.base[colA[4 * t + r] * sb.ld + sb.row] = cx<T>{cre[t][r], cim[t][r]};
    }
    if (more) {
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = nv[u];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_jac_rot(JacBatch jb, int step, int part) {
  const int pi = blockIdx.z;
  if (pi >= jb.count) return;
  const JacProb P = jb.p[pi];
  if (step >= P.nblk - 1 || (int)blockIdx.x >= P.nblk / 2) return;
  if (P.st->active == 0) return;
  if (P.pflag[blockIdx.x] == 0) return;
  const int nv = P.V ? P.ncol : 0;
  const int rows = (part == 1) ? P.m : P.m + nv;
  const int c0 = (part == 2 ? P.m : 0) + blockIdx.y * RRC;
  if (c0 >= rows) return;
  const int c1 = min(rows, c0 + RRC);
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
// The same Gram and rotation with every real product on three BF16 MFMAs
// (mfma.h); K = 32 per instruction covers a whole panel width.
__global__ __launch_bounds__(256) void k_jac_gram_bf16(JacBatch jb, int step) {
  const int pi = blockIdx.z;
  if (pi >= jb.count) return;
  const JacProb P = jb.p[pi];
  if (step >= P.nblk - 1 || (int)blockIdx.x >= P.nblk / 2) return;
  if (P.st->active == 0) return;
  const int r0 = blockIdx.y * GRC;
  if (r0 >= P.m) return;
  const int r1 = min(P.m, r0 + GRC);
  int bi, bj;
  rr_pair2(P.nblk, step, blockIdx.x, bi, bj);
  if (pair_unchanged(P, bi, bj)) return;
  // A 64-row slab, split once as it is staged: Sh[part][column][row] with
  // parts re_hi, re_lo, im_hi, im_lo, transposed so that a lane's 8
  // consecutive rows of one column (its MFMA operand) are one 16-byte read.
  __shared__ __attribute__((aligned(16))) __bf16 Sh[4][32][72];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int I = wave >> 1, J = wave & 1, g8 = (lane >> 4) * 8;
  const cx<float>* A = (const cx<float>*)P.A;
  double gr[4] = {0, 0, 0, 0}, gi[4] = {0, 0, 0, 0};
  // the next 64-row slab is loaded into registers while this one is multiplied
  cx<float> nxt[8];
  auto fetch = [&](int s0) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int c = wave + 4 * u;
      nxt[u] = cx<float>{0, 0};
      if (s0 + lane < r1) nxt[u] = A[(size_t)panel_col(bi, bj, c) * P.lda + s0 + lane];
    }
  };
  auto op = [&](int part, int c, int k) -> v8bf { return *(const v8bf*)&Sh[part][c][k]; };
  fetch(r0);
  for (int s0 = r0; s0 < r1; s0 += 64) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int c = wave + 4 * u;
      const __bf16 rh = (__bf16)nxt[u].re, ih = (__bf16)nxt[u].im;
      Sh[0][c][lane] = rh;
      Sh[1][c][lane] = (__bf16)(nxt[u].re - (float)rh);
      Sh[2][c][lane] = ih;
      Sh[3][c][lane] = (__bf16)(nxt[u].im - (float)ih);
    }
    __syncthreads();
    if (s0 + 64 < r1) fetch(s0 + 64);
    v4f are = {0, 0, 0, 0}, aim = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < 64; kk += 32) {
      const int cx_ = I * 16 + (lane & 15), cy = J * 16 + (lane & 15), k = kk + g8;
      const Split8 xr{op(0, cx_, k), op(1, cx_, k)}, xi{op(2, cx_, k), op(3, cx_, k)};
      const Split8 xn{-xi.hi, -xi.lo};
      const Split8 yr{op(0, cy, k), op(1, cy, k)}, yi{op(2, cy, k), op(3, cy, k)};
      // conj(x) y
      are = mma3_bf16(xr, yr, are);
      are = mma3_bf16(xi, yi, are);
      aim = mma3_bf16(xr, yi, aim);
      aim = mma3_bf16(xn, yr, aim);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      gr[r] += (double)are[r];
      gi[r] += (double)aim[r];
    }
    __syncthreads();
  }
  cx<double>* out = P.gpart + ((size_t)blockIdx.x * P.ngchunk + blockIdx.y) * 1024;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = I * 16 + MF<float>::row(lane, r), j = J * 16 + (lane & 15);
    out[i * 32 + j] = cx<double>{gr[r], gi[r]};
  }
}

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
__global__ __launch_bounds__(256) void k_jac_rot_mixed(JacBatch jb, int step, int ny_theta) {
  const int pi = blockIdx.z;
  if (pi >= jb.count) return;
  const JacProb P = jb.p[pi];
  if (step >= P.nblk - 1 || (int)blockIdx.x >= P.nblk / 2) return;
  if (P.st->active == 0) return;
  if (P.pflag[blockIdx.x] == 0) return;
  const bool theta = (int)blockIdx.y < ny_theta;
  int c0, c1;
  if (theta) {
    c0 = blockIdx.y * RRC;
    if (c0 >= P.m) return;
    c1 = min(P.m, c0 + RRC);
  } else {
    const int nv = P.V ? P.ncol : 0;
    c0 = P.m + (blockIdx.y - ny_theta) * RRC;
    if (c0 >= P.m + nv) return;
    c1 = min(P.m + nv, c0 + RRC);
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

// Newton-Schulz step toward the polar factor in FP64: S <- (3 I - S) / 2.
__global__ void k_ns_coef(cx<double>* S, int n) {
  const size_t tot = (size_t)n * n;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
    const size_t i = e / n, j = e - i * n;
    const cx<double> v = S[e];
    S[e] = cx<double>{((i == j) ? 1.5 : 0.0) - 0.5 * v.re, -0.5 * v.im};
  }
}

void launch_ns_coef(cx<double>* S, int n, hipStream_t s) {
  size_t g = ((size_t)n * n + 255) / 256;
  g = g < 1 ? 1 : (g > 2048 ? 2048 : g);
  hipLaunchKernelGGL(k_ns_coef, dim3((unsigned)g), dim3(256), 0, s, S, n);
}

template <typename T>
void launch_jac_gram(const JacBatch& b, int maxpairs, int maxgch, int step, int bf16, hipStream_t s) {
  if (bf16)
    hipLaunchKernelGGL(k_jac_gram_bf16, dim3(maxpairs, maxgch, b.count), dim3(256), 0, s, b, step);
  else
    hipLaunchKernelGGL(k_jac_gram<T>, dim3(maxpairs, maxgch, b.count), dim3(256), 0, s, b, step);
}
template <typename T>
void launch_jac_evd(const JacBatch& b, int maxpairs, int step, int inner_sweeps, int stamp, hipStream_t s) {
  hipLaunchKernelGGL(k_jac_evd<T>, dim3(maxpairs, b.count), dim3(256), 0, s, b, step, inner_sweeps, stamp);
}
template <typename T>
void launch_jac_rot(const JacBatch& b, int maxpairs, int maxrch_a, int maxrch_v, int step, int mode, hipStream_t s) {
  if (mode == ROT_MIXED)
    hipLaunchKernelGGL(k_jac_rot_mixed, dim3(maxpairs, maxrch_a + maxrch_v, b.count), dim3(256), 0, s, b, step,
                       maxrch_a);
  else
    hipLaunchKernelGGL(k_jac_rot<T>, dim3(maxpairs, maxrch_a + maxrch_v, b.count), dim3(256), 0, s, b, step, 0);
}
template <>
void launch_jac_gram<double>(const JacBatch& b, int maxpairs, int maxgch, int step, int, hipStream_t s) {
  hipLaunchKernelGGL(k_jac_gram<double>, dim3(maxpairs, maxgch, b.count), dim3(256), 0, s, b, step);
}
template <>
void launch_jac_rot<double>(const JacBatch& b, int maxpairs, int maxrch_a, int maxrch_v, int step, int,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_jac_rot<double>, dim3(maxpairs, maxrch_a + maxrch_v, b.count), dim3(256), 0, s, b, step, 0);
}
template void launch_jac_gram<float>(const JacBatch&, int, int, int, int, hipStream_t);
template void launch_jac_rot<float>(const JacBatch&, int, int, int, int, int, hipStream_t);
template void launch_jac_evd<float>(const JacBatch&, int, int, int, int, hipStream_t);
template void launch_jac_evd<double>(const JacBatch&, int, int, int, int, hipStream_t);

}  // namespace mpo

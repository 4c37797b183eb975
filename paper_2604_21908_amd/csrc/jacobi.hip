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
//               at most one or two sweeps of cyclic Jacobi on G (FP64
//               angles; rotations in the working precision: FP64, or FP32 for
//               the FP32 and mixed forms; the outer iteration finishes what
//               they leave), and D = W - I rounded to the working precision
//   k_jac_rot   P <- P + P D (rotation.hip)
//   k_jac_gram_bf16  the mixed form's Gram matrices with split-BF16 products
//               (the EVD stays FP64)
//   k_ns_corr   the Newton-Schulz correction of the mixed form's rotations
#include "common.h"
#include "mfma.h"

namespace mpo {

// Inner cyclic-Jacobi sweeps per panel EVD (a kernel argument): two already
// give the outer iteration its full convergence rate, more only add latency;
// one costs about one extra outer sweep but halves the EVD.

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
    // conj(x) y as three real products (Gauss): k1 = xr yr, k2 = xi yi,
    // k3 = (xr - xi)(yr + yi); Re = k1 + k2, Im = k3 - k1 + k2 (formed in FP64
    // from the slab's FP32 or FP64 sums) -- three MFMA chains instead of four
    acc_t k1 = {0, 0, 0, 0}, k2 = {0, 0, 0, 0}, k3 = {0, 0, 0, 0};
#pragma unroll 4
    for (int kk = 0; kk < 64; kk += 4) {
      const cx<T> x = Pc[kk + (lane >> 4)][I * 16 + (lane & 15)];   // A = P^dag: conj applied below
      const cx<T> y = Pc[kk + (lane >> 4)][J * 16 + (lane & 15)];
      k1 = MF<T>::mma(x.re, y.re, k1);
      k2 = MF<T>::mma(x.im, y.im, k2);
      k3 = MF<T>::mma(x.re - x.im, y.re + y.im, k3);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double a1 = (double)k1[r], a2 = (double)k2[r];
      gr[r] += a1 + a2;
      gi[r] += ((double)k3[r] - a1) + a2;
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
// Hardware reciprocal and reciprocal square root estimates (FP64, positive
// normal arguments, about 2^-23 relative) refined by Newton steps, each of
// which squares the relative error: one step leaves about 2^-45, two a few
// ulp.
__device__ __forceinline__ double rcp_nr1(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  return fma(y, fma(-x, y, 1.0), y);
}
__device__ __forceinline__ double rsq_nr1(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  return fma(0.5 * y, fma(-x * y, y, 1.0), y);
}
__device__ __forceinline__ double rsq_nr2(double x) {
  const double y = rsq_nr1(x);
  return fma(0.5 * y, fma(-x * y, y, 1.0), y);
}

// Complex Jacobi rotation of pair (p, q) of the Hermitian G:
// J = [[c, z], [-conj(z), c]], z = tau c, c = 1 / sqrt(1 + |tau|^2), with the
// complex tangent tau = t g_pq / |g_pq| and t the smaller root of
// t^2 + 2 zeta t - 1 = 0, zeta = (g_qq - g_pp) / (2 |g_pq|); it zeroes the
// (p, q) entry of J^dag G J.  Only c needs full accuracy: c^2 + |z|^2 = 1
// holds for whatever tau is used, so tau (which only sets how well the entry
// is zeroed) comes from cheaper estimates.  Returns false (c = 1, z = 0)
// when |g_pq| is below tol sqrt(g_pp g_qq).  Branch-free: evaluated for every
// lane, the identity selected where no rotation applies.
// FINE: the once-refined estimates for 1 / |g_pq|, sqrt(1 + zeta^2) and the
// tangent (about 2^-45: the FP64 form, whose tolerance is near FP64 rounding);
// otherwise the bare hardware estimates (about 2^-23), enough to zero the
// entry to well below the FP32 and mixed forms' tolerances.  c is fully
// refined either way.
template <bool FINE>
__device__ __forceinline__ double est_rsq(double x) {
  return FINE ? rsq_nr1(x) : __builtin_amdgcn_rsq(x);
}
template <bool FINE>
__device__ __forceinline__ double est_rcp(double x) {
  return FINE ? rcp_nr1(x) : __builtin_amdgcn_rcp(x);
}
template <bool FINE>
__device__ __forceinline__ bool jac_angle(double app, double aqq, cx<double> g, double tol, double& c, double& zr,
                                          double& zi) {
  const double g2 = g.re * g.re + g.im * g.im;
  const bool rot = (g2 > 0.0) & (g2 > tol * tol * fmax(app * aqq, 0.0));
  const double g2s = rot ? g2 : 1.0;
  const double rm = est_rsq<FINE>(g2s);                // ~ 1 / |g_pq|
  const double zeta = 0.5 * (aqq - app) * rm;
  const double az = fabs(zeta);
  // 1 / (|zeta| + sqrt(1 + zeta^2)); for |zeta| > 2^60 the root is |zeta| to
  // working precision and zeta^2 could overflow
  const bool big = az > 0x1p60;
  const double z1 = big ? 1.0 : 1.0 + zeta * zeta;
  const double h = z1 * est_rsq<FINE>(z1);
  const double ta = est_rcp<FINE>(big ? az : az + h) * (big ? 0.5 : 1.0);
  const double t = zeta >= 0.0 ? ta : -ta;
  // the phase g_pq / |g_pq| first (|g_pq| may be near the underflow limit,
  // its reciprocal near overflow), then tau = t e and |tau|^2 = t^2 |e|^2
  const double er = g.re * rm, ei = g.im * rm;
  const double cv = rsq_nr2(fma(t * t, er * er + ei * ei, 1.0));
  const double sv = t * cv;
  c = rot ? cv : 1.0;
  zr = rot ? sv * er : 0.0;
  zi = rot ? sv * ei : 0.0;
  return rot;
}

template <typename E>
__device__ __forceinline__ bool jac_angle_e(E app, E aqq, cx<E> g, double tol, bool fine, E& c, E& zr, E& zi);
template <>
__device__ __forceinline__ bool jac_angle_e<double>(double app, double aqq, cx<double> g, double tol, bool fine,
                                                    double& c, double& zr, double& zi) {
  return fine ? jac_angle<true>(app, aqq, g, tol, c, zr, zi) : jac_angle<false>(app, aqq, g, tol, c, zr, zi);
}
// FP32 panels (the FP32 and mixed forms): the angle from the FP32 entries in
// FP64 arithmetic (the squares of tiny entries would be denormal in FP32),
// the rotation itself applied in FP32.
template <>
__device__ __forceinline__ bool jac_angle_e<float>(float app, float aqq, cx<float> g, double tol, bool, float& c,
                                                   float& zr, float& zi) {
  double cd, zrd, zid;
  const bool rot = jac_angle<false>((double)app, (double)aqq, cx<double>{(double)g.re, (double)g.im}, tol, cd, zrd, zid);
  c = (float)cd;
  zr = (float)zrd;
  zi = (float)zid;
  return rot;
}

// In a round-robin step the 32 indices form 16 disjoint pairs; the rotation
// J_k of pair k acts on columns (p_k, q_k).  Thread (kr, kc) owns the 2x2
// block of G at rows (p_kr, q_kr) x columns (p_kc, q_kc) and replaces it by
// J_kr^dag G_block J_kc, and likewise W's rows (p_kr, q_kr) x columns
// (p_kc, q_kc) by W_block J_kc: every entry is written by exactly one thread.
// Every lane computes the angle of its own column pair kc from the round's G;
// the row pair's angle comes from the lane of the same wave whose kc equals kr.
// G is double-buffered (read one copy, write the other), so a round needs a
// single barrier; W is updated in place (each thread touches only its block).
// The pairs of the 31 rounds are tabulated once as LDS byte offsets.
// E is the arithmetic of the rotations: FP64 in the FP64 form, FP32 in the
// FP32 and mixed forms (whose tolerances are far above FP32 rounding); the
// partial Gram matrices are summed in FP64 either way, angles formed in FP64.
constexpr int EVD_LD = 33;                       // row stride of G and W (entries)
template <typename T, typename E>
__global__ __launch_bounds__(256) void k_jac_evd(JacBatch jb, int step, int inner_sweeps) {
  constexpr int EVD_ROWB = EVD_LD * (int)sizeof(cx<E>);   // ... in bytes
  const int pi = blockIdx.y;
  if (pi >= jb.count) return;
  const JacProb P = jb.p[pi];
  if (step >= P.nblk - 1 || (int)blockIdx.x >= P.nblk / 2) return;
  const double tol = P.tol;
  __shared__ cx<E> G[2][32][EVD_LD];
  __shared__ cx<E> W[32][EVD_LD];
  __shared__ ushort4 ptab[31][16];   // pair k of round st: (p, q) row and column byte offsets
  __shared__ int flag, anyrot;
  const int tid = threadIdx.x;
  const int gi = tid >> 3, gj0 = (tid & 7) * 4;
  int* pflag = P.pflag + blockIdx.x;
  int bi, bj;
  rr_pair2(P.nblk, step, blockIdx.x, bi, bj);
  // Every load of the set-up is issued before any of them is tested: the
  // state flag, the pair-skip stamps and all partial Gram matrices (read even
  // for a pair that turns out skipped; their sum is then discarded).
  const int active = P.st->active;
  const int stamp = P.st->epoch * P.nblk + step + 1;
  const int chk = P.pchk[bi * P.nblk + bj], mod_i = P.bmod[bi], mod_j = P.bmod[bj];
  const int nch = (P.m + GRC - 1) / GRC;
  const cx<double>* gp = P.gpart + (size_t)blockIdx.x * P.ngchunk * 1024 + gi * 32 + gj0;
  double sr[4] = {0, 0, 0, 0}, si[4] = {0, 0, 0, 0};
  for (int c0 = 0; c0 < nch; c0 += 8) {
    cx<double> v[8][4];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const size_t off = (size_t)min(c0 + c, nch - 1) * 1024;   // clamped, masked below
#pragma unroll
      for (int u = 0; u < 4; ++u) v[c][u] = gp[off + u];
    }
    // in chunk order (deterministic); a clamped duplicate adds zero
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const double w = (c0 + c < nch) ? 1.0 : 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        sr[u] += w * v[c][u].re;
        si[u] += w * v[c][u].im;
      }
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    G[0][gi][gj0 + u] = cx<E>{(E)sr[u], (E)si[u]};
    W[gi][gj0 + u] = cx<E>{(E)((gi == gj0 + u) ? 1 : 0), (E)0};
  }
  for (int e = tid; e < 31 * 16; e += 256) {
    int p, q;
    rr_pair2(32, e >> 4, e & 15, p, q);
    ptab[e >> 4][e & 15] = ushort4{(unsigned short)(p * EVD_ROWB), (unsigned short)(q * EVD_ROWB),
                                   (unsigned short)(p * sizeof(cx<E>)), (unsigned short)(q * sizeof(cx<E>))};
  }
  if (active == 0) return;
  if (chk > 0 && chk > mod_i && chk > mod_j) {   // unchanged converged pair
    if (tid == 0) *pflag = 0;
    return;
  }
  if (tid == 0) {
    flag = 0;
    anyrot = 0;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = gj0 + u;
    if (j > gi) {
      // on the entries as the rotations see them, in FP64 (as jac_angle tests)
      const cx<E> g = G[0][gi][j];
      const double d = (double)G[0][gi][gi].re * (double)G[0][j][j].re;
      const double g2 = (double)g.re * (double)g.re + (double)g.im * (double)g.im;
      if (d > 0 && g2 > tol * tol * d) flag = 1;
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
  const int src = (tid & 48) | kr;   // lane of this wave with kc == kr
  char* const g0 = (char*)&G[0][0][0];
  char* const wb = (char*)&W[0][0];
  int cur = 0;
  for (int isw = 0; isw < inner_sweeps; ++isw) {
    for (int st = 0; st < 31; ++st) {
      char* const gc = g0 + cur * (32 * EVD_ROWB);
      char* const gn = g0 + (cur ^ 1) * (32 * EVD_ROWB);
      const ushort4 R = ptab[st][kr], C = ptab[st][kc];
      auto at = [](char* base, int off) -> cx<E>& { return *(cx<E>*)(base + off); };
      const cx<E> a00 = at(gc, R.x + C.z), a01 = at(gc, R.x + C.w), a10 = at(gc, R.y + C.z),
                  a11 = at(gc, R.y + C.w);
      const cx<E> w00 = at(wb, R.x + C.z), w01 = at(wb, R.x + C.w), w10 = at(wb, R.y + C.z),
                  w11 = at(wb, R.y + C.w);
      // column pair's own entries: (p, p) at row p col p, (q, q), (p, q)
      const E app = at(gc, C.x + C.z).re, aqq = at(gc, C.y + C.w).re;
      const cx<E> gpq = at(gc, C.x + C.w);
      E cc, zcr, zci;
      const bool rot = jac_angle_e<E>(app, aqq, gpq, tol, sizeof(T) == 8, cc, zcr, zci);
      // A round in which none of the 16 pairs rotates would rewrite G and W
      // unchanged: skipped, with no barrier and no buffer swap.  Every wave
      // holds all 16 column pairs (kc = lane & 15) and reads the same G, so all
      // waves take the same decision.
      if (!__any(rot)) continue;
      if (rot) anyrot = isw + 1;
      const E cr = __shfl(cc, src, 64), zrr = __shfl(zcr, src, 64), zri = __shfl(zci, src, 64);
      // H = G_block J_c; x * (-conj(zc)) = -(x.re zcr + x.im zci) + i (x.re zci - x.im zcr)
      const E h00r = a00.re * cc - (a01.re * zcr + a01.im * zci);
      const E h00i = a00.im * cc + (a01.re * zci - a01.im * zcr);
      const E h01r = a00.re * zcr - a00.im * zci + a01.re * cc;
      const E h01i = a00.re * zci + a00.im * zcr + a01.im * cc;
      const E h10r = a10.re * cc - (a11.re * zcr + a11.im * zci);
      const E h10i = a10.im * cc + (a11.re * zci - a11.im * zcr);
      const E h11r = a10.re * zcr - a10.im * zci + a11.re * cc;
      const E h11i = a10.re * zci + a10.im * zcr + a11.im * cc;
      // G' = J_r^dag H, J_r^dag = [[cr, -zr], [conj(zr), cr]]
      at(gn, R.x + C.z) = cx<E>{cr * h00r - (zrr * h10r - zri * h10i), cr * h00i - (zrr * h10i + zri * h10r)};
      at(gn, R.x + C.w) = cx<E>{cr * h01r - (zrr * h11r - zri * h11i), cr * h01i - (zrr * h11i + zri * h11r)};
      at(gn, R.y + C.z) = cx<E>{zrr * h00r + zri * h00i + cr * h10r, zrr * h00i - zri * h00r + cr * h10i};
      at(gn, R.y + C.w) = cx<E>{zrr * h01r + zri * h01i + cr * h11r, zrr * h01i - zri * h01r + cr * h11i};
      if (!(zcr == (E)0 && zci == (E)0)) {
        // W' = W_block J_c on rows (pr, qr)
        at(wb, R.x + C.z) =
            cx<E>{w00.re * cc - (w01.re * zcr + w01.im * zci), w00.im * cc + (w01.re * zci - w01.im * zcr)};
        at(wb, R.x + C.w) =
            cx<E>{w00.re * zcr - w00.im * zci + w01.re * cc, w00.re * zci + w00.im * zcr + w01.im * cc};
        at(wb, R.y + C.z) =
            cx<E>{w10.re * cc - (w11.re * zcr + w11.im * zci), w10.im * cc + (w11.re * zci - w11.im * zcr)};
        at(wb, R.y + C.w) =
            cx<E>{w10.re * zcr - w10.im * zci + w11.re * cc, w10.re * zci + w10.im * zcr + w11.im * cc};
      }
      __syncthreads();
      cur ^= 1;
    }
    // anyrot only grows and is isw + 1 or more iff some pair rotated in this
    // sweep; every thread reads it after the barrier of the sweep's last
    // rotating round (a skipped round writes nothing)
    if (anyrot <= isw) break;
  }
  // D = W - I, rounded entry by entry (see k_jac_rot)
  cx<T>* D = (cx<T>*)P.dmat + (size_t)blockIdx.x * 1024;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = gi, c = gj0 + u;
    D[r * 32 + c] = cx<T>{(T)(W[r][c].re - (E)(r == c ? 1 : 0)), (T)W[r][c].im};
  }
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
  const bool mirror = I == 1 && J == 0;
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
    // block (1, 0) is the conjugate transpose of block (0, 1): its wave only
    // stages
    if (!mirror) {
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
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      gr[r] += (double)are[r];
      gi[r] += (double)aim[r];
    }
    __syncthreads();
  }
  cx<double>* out = P.gpart + ((size_t)blockIdx.x * P.ngchunk + blockIdx.y) * 1024;
  if (mirror) return;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = I * 16 + MF<float>::row(lane, r), j = J * 16 + (lane & 15);
    out[i * 32 + j] = cx<double>{gr[r], gi[r]};
    if (I != J) out[j * 32 + i] = cx<double>{gr[r], -gi[r]};
  }
}

// Newton-Schulz step toward the polar factor, W <- W + W (I - W^dag W) / 2
// in the transposed row-major storage X = W^T: X <- X + E X with
// E = (I - S) / 2, S = X X^dag (FP64, only its upper tiles computed; the
// lower ones are the conjugates).  E, of the size of the drift from
// unitarity, is rounded to the working precision T.
template <typename T>
__global__ void k_ns_corr(const cx<double>* S, cx<T>* E, int n) {
  const size_t tot = (size_t)n * n;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e - (size_t)i * n);
    cx<double> v = S[e];
    if (i / GEMM_TILE > j / GEMM_TILE) {
      const cx<double> u = S[(size_t)j * n + i];
      v = cx<double>{u.re, -u.im};
    }
    E[e] = cx<T>{(T)(0.5 * ((i == j ? 1.0 : 0.0) - v.re)), (T)(-0.5 * v.im)};
  }
}

template <typename T>
void launch_ns_corr(const cx<double>* S, cx<T>* E, int n, hipStream_t s) {
  size_t g = ((size_t)n * n + 255) / 256;
  g = g < 1 ? 1 : (g > 2048 ? 2048 : g);
  hipLaunchKernelGGL(k_ns_corr<T>, dim3((unsigned)g), dim3(256), 0, s, S, E, n);
}

template <typename T>
void launch_jac_gram(const JacBatch& b, int maxpairs, int maxgch, int step, int bf16, hipStream_t s) {
  if (bf16)
    hipLaunchKernelGGL(k_jac_gram_bf16, dim3(maxpairs, maxgch, b.count), dim3(256), 0, s, b, step);
  else
    hipLaunchKernelGGL(k_jac_gram<T>, dim3(maxpairs, maxgch, b.count), dim3(256), 0, s, b, step);
}
template <typename T>
void launch_jac_evd(const JacBatch& b, int maxpairs, int step, int inner_sweeps, hipStream_t s) {
  // rotations in the working precision: FP32 in the FP32 and mixed forms
  hipLaunchKernelGGL((k_jac_evd<T, T>), dim3(maxpairs, b.count), dim3(256), 0, s, b, step, inner_sweeps);
}
template <>
void launch_jac_gram<double>(const JacBatch& b, int maxpairs, int maxgch, int step, int, hipStream_t s) {
  hipLaunchKernelGGL(k_jac_gram<double>, dim3(maxpairs, maxgch, b.count), dim3(256), 0, s, b, step);
}
template void launch_jac_gram<float>(const JacBatch&, int, int, int, int, hipStream_t);
template void launch_jac_evd<float>(const JacBatch&, int, int, int, hipStream_t);
template void launch_jac_evd<double>(const JacBatch&, int, int, int, hipStream_t);
template void launch_ns_corr<float>(const cx<double>*, cx<float>*, int, hipStream_t);
template void launch_ns_corr<double>(const cx<double>*, cx<double>*, int, hipStream_t);

}  // namespace mpo

// Householder QR preconditioner of the Jacobi SVD (gfx950).
//
// The bond matrix enters as M = (lambda theta)^dag, n x m column-major.  Its
// QR factorisation M = Q R gives theta = L Q^dag with L = R^dag lower
// trapezoidal; one-sided Jacobi on the columns of L then needs far fewer
// sweeps than on theta itself (the QR-preconditioned Jacobi SVD of Drmac and
// Veselic), and the right singular vectors of theta are V = Q [W; 0] with W
// the accumulated Jacobi rotations -- no division by singular values.
//
//   k_qr_panel   up to 16 workgroups factor a QNB-column panel (complex
//                Householder reflectors, LAPACK's sign convention,
//                right-looking, rows in FP64 registers, FP64 sums across the
//                workgroups) and build the upper-triangular T of the compact
//                WY form
//   k_qr_w1/w2/upd  C <- (I - V op(T) V^dag) C: row-chunked partial products
//                V^dag C, their FP64 sum times op(T), the rank-QNB update; the
//                trailing update (op = dag) and the formation of V (op = identity)
//   k_lower_from_r  L = R^dag into the column-major Jacobi operand
//   k_build_y / k_vh_rows   [W_k; 0] and B_{i+1} <- V_k^dag, lambda_i <- s_<k
#include "common.h"
#include "mfma.h"

namespace mpo {

constexpr int QPN = 4096;   // largest panel height: n <= 4 chi_max

// V (rows [p0, n), nb columns) at row i, column a of the panel at p0; zero
// unless `ok`.  The load always goes to a valid address (row and column
// clamped) and the value is selected afterwards, so that a thread's loads
// are issued together rather than each behind a branch.
template <typename T>
__device__ __forceinline__ cx<T> v_entry(const cx<T>* M, int n, int p0, int nb, int i, int a, bool ok) {
  const int ac = min(a, nb - 1);
  const int ic = min(max(i, p0 + ac), n - 1);
  const cx<T> t = M[(size_t)(p0 + ac) * n + ic];
  const bool live = ok && a < nb && i < n;
  // the loaded value is always used (times a 0/1 mask), so the compiler
  // cannot sink the load behind a branch
  const T below = (live && i > p0 + a) ? (T)1 : (T)0;
  const T diag = (live && i == p0 + a) ? (T)1 : (T)0;
  return cx<T>{below * t.re + diag, below * t.im};
}

// Partial products V^dag C over the QRC1 rows of chunk blockIdx.y, for the
// QAT columns of tile blockIdx.x: 128-row slabs staged in LDS (coalesced),
// each wave multiplies 32 rows per slab on MFMA; the four wave sums are added
// in FP64 and stored to wpart[chunk].
template <typename T>
__global__ __launch_bounds__(256) void k_qr_w1(QrApplyBatch ab, int p0) {
  const int pi = blockIdx.z;
  if (pi >= ab.count) return;
  const QrApplyProb P = ab.p[pi];
  if (p0 >= P.r) return;
  const int cbeg = P.c0 + blockIdx.x * QAT;
  if (cbeg >= P.c1) return;
  const int n = P.n;
  const int rbeg = p0 + blockIdx.y * QRC1;
  if (rbeg >= n) return;
  const int rend = min(n, rbeg + QRC1);
  const int nb = min(QNB, P.r - p0);
  const int ncols = min(QAT, P.c1 - cbeg);
  const cx<T>* M = (const cx<T>*)P.M;
  const cx<T>* C = (const cx<T>*)P.C;
  typedef typename MF<T>::acc acc_t;
  __shared__ cx<T> Vs[128][QNB + 1];
  __shared__ cx<T> Cs[128][QAT + 1];
  __shared__ double Wp[4][QNB][QAT][2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  acc_t wre = {0, 0, 0, 0}, wim = {0, 0, 0, 0};
  for (int r0 = rbeg; r0 < rend; r0 += 128) {
    static_assert((128 * QNB) % 256 == 0 && (128 * QAT) % 256 == 0, "whole staging rounds");
#pragma unroll
    for (int j = 0; j < 128 * QNB / 256; ++j) {
      const int e = tid + 256 * j;
      const int rr = e % 128, a = e / 128, i = r0 + rr;
      Vs[rr][a] = v_entry(M, n, p0, nb, i, a, i < rend);
    }
#pragma unroll
    for (int j = 0; j < 128 * QAT / 256; ++j) {
      const int e = tid + 256 * j;
      const int rr = e % 128, c = e / 128, i = r0 + rr;
      const cx<T> v = C[(size_t)(cbeg + min(c, ncols - 1)) * P.ldc + min(i, rend - 1)];   // clamped, masked
      const T mk = (i < rend && c < ncols) ? (T)1 : (T)0;
      Cs[rr][c] = cx<T>{mk * v.re, mk * v.im};
    }
    __syncthreads();
#pragma unroll
    for (int kk = wave * 32; kk < wave * 32 + 32; kk += 4) {
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
  const int a = tid / QAT, c = tid % QAT;
  if (c < ncols) {
    cx<double>* out = (cx<double>*)P.wpart + ((size_t)blockIdx.y * QNB + a) * P.ldp + cbeg + c;
    *out = cx<double>{Wp[0][a][c][0] + Wp[1][a][c][0] + Wp[2][a][c][0] + Wp[3][a][c][0],
                      Wp[0][a][c][1] + Wp[1][a][c][1] + Wp[2][a][c][1] + Wp[3][a][c][1]};
  }
}

// w2 = op(T) * (sum of the chunk partials, in chunk order), one 16 x QAT tile
// per workgroup.
template <typename T>
__global__ __launch_bounds__(256) void k_qr_w2(QrApplyBatch ab, int p0) {
  const int pi = blockIdx.y;
  if (pi >= ab.count) return;
  const QrApplyProb P = ab.p[pi];
  if (p0 >= P.r) return;
  const int cbeg = P.c0 + blockIdx.x * QAT;
  if (cbeg >= P.c1) return;
  const int ncols = min(QAT, P.c1 - cbeg);
  const int nch = (P.n - p0 + QRC1 - 1) / QRC1;
  const cx<T>* Tf = (const cx<T>*)P.Tf + (size_t)(p0 / QNB) * QNB * QNB;
  __shared__ cx<double> Tl[QNB][QNB];
  __shared__ cx<double> W1[QNB][QAT + 1];
  const int tid = threadIdx.x;
  const int a = tid / QAT, c = tid % QAT;
  if (ab.conj_t) {
    const cx<T> u = Tf[c * QNB + a];
    Tl[a][c] = cx<double>{(double)u.re, -(double)u.im};
  } else {
    const cx<T> t = Tf[a * QNB + c];
    Tl[a][c] = cx<double>{(double)t.re, (double)t.im};
  }
  double sr = 0, si = 0;
  if (c < ncols) {
    const cx<double>* wp = (const cx<double>*)P.wpart + (size_t)a * P.ldp + cbeg + c;
    for (int ch = 0; ch < nch; ++ch) {
      const cx<double> v = wp[(size_t)ch * QNB * P.ldp];
      sr += v.re;
      si += v.im;
    }
  }
  W1[a][c] = cx<double>{sr, si};
  __syncthreads();
  if (c < ncols) {
    double yr = 0, yi = 0;
    for (int b = 0; b < QNB; ++b) {
      const cx<double> t = Tl[a][b], u = W1[b][c];
      yr += t.re * u.re - t.im * u.im;
      yi += t.re * u.im + t.im * u.re;
    }
    ((cx<T>*)P.w2)[(size_t)a * P.ldp + cbeg + c] = cx<T>{(T)yr, (T)yi};
  }
}

// C <- C - V w2 on QRC2 rows (chunk blockIdx.y) x QAT columns (tile
// blockIdx.x), on MFMA in the transposed orientation C^T -= w2^T V^T: each
// 16-lane group covers 16 consecutive rows of one column of C; each wave
// takes 64 rows as four 16-row strips.
template <typename T>
__global__ __launch_bounds__(256) void k_qr_upd(QrApplyBatch ab, int p0) {
  const int pi = blockIdx.z;
  if (pi >= ab.count) return;
  const QrApplyProb P = ab.p[pi];
  if (p0 >= P.r) return;
  const int cbeg = P.c0 + blockIdx.x * QAT;
  if (cbeg >= P.c1) return;
  const int n = P.n;
  const int rbeg = p0 + blockIdx.y * QRC2;
  if (rbeg >= n) return;
  const int nb = min(QNB, P.r - p0);
  const int ncols = min(QAT, P.c1 - cbeg);
  const cx<T>* M = (const cx<T>*)P.M;
  cx<T>* C = (cx<T>*)P.C;
  typedef typename MF<T>::acc acc_t;
  __shared__ cx<T> W2[QNB][QAT + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  {
    const int a = tid / QAT, c = tid % QAT;
    const cx<T> w = ((const cx<T>*)P.w2)[(size_t)a * P.ldp + cbeg + min(c, ncols - 1)];   // clamped, masked
    const T mk = c < ncols ? (T)1 : (T)0;
    W2[a][c] = cx<T>{mk * w.re, mk * w.im};
  }
  // every load of the workgroup first (C may alias M, so loads are not moved
  // past the stores by the compiler), then the products, then the stores
  cx<T> cv[4][4], vv[4][QNB / 4];
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int i = rbeg + wave * 64 + st * 16 + (lane & 15);
    const bool valid = i < n && i < rbeg + QRC2;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = MF<T>::row(lane, r);
      const cx<T> v = C[(size_t)(cbeg + min(c, ncols - 1)) * P.ldc + min(i, n - 1)];   // clamped, masked
      const T mk = (valid && c < ncols) ? (T)1 : (T)0;
      cv[st][r] = cx<T>{mk * v.re, mk * v.im};
    }
#pragma unroll
    for (int kq = 0; kq < QNB / 4; ++kq) vv[st][kq] = v_entry(M, n, p0, nb, i, 4 * kq + (lane >> 4), valid);
  }
  __syncthreads();
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int i = rbeg + wave * 64 + st * 16 + (lane & 15);
    const bool valid = i < n && i < rbeg + QRC2;
    acc_t cre, cim;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      cre[r] = cv[st][r].re;
      cim[r] = cv[st][r].im;
    }
#pragma unroll
    for (int kq = 0; kq < QNB / 4; ++kq) {
      const int a = 4 * kq + (lane >> 4);
      const cx<T> v = vv[st][kq];
      const cx<T> w = W2[a][lane & 15];   // A[c][a] = w2[a][c], negated for the subtraction
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
// Panel factorisation over several workgroups.  Workgroup w holds panel rows [256 w, 256 w + 256), one
// per thread, all QNB columns in FP64 registers, and the columns are factored
// right-looking.  Column j needs the tail norm |x_{>j}|^2 and alpha = x_j
// (summed over the problem's workgroups; every workgroup then forms the same
// reflector, LAPACK's complex Householder as in k_qr_panel, and scales its
// rows of v_j), then one more sum: w_k = v_j^dag a_k (k > j) and
// z_q = v_q^dag v_j (q < j), after which a_k <- a_k - c_k v_j with
// c_k = conj(tau_j) w_k (H_j^dag from the left) and
// T[0:j, j] = -tau_j T[0:j, 0:j] z.  The second sum also carries, for column
// j + 1, A = |a_{j+1}|^2, B = a_{j+1}^dag v_j, C = |v_j|^2 over the rows below
// j + 1 and the row-(j + 1) entries, so that its tail norm
// A - 2 Re(c B) + |c|^2 C and alpha come without a sum of their own; when the
// expansion could lose more than about one digit to cancellation
// (result < 1/10 of A + 2|c||B| + |c|^2 C) the norm is summed exactly
// instead (a rank-deficient panel takes a few such sums; a generic one none
// after its first column).  Sums run per wave, over waves in order, then over workgroups in
// order, so every workgroup gets the same bits and takes the same decisions.
// A barrier is a counter every workgroup increments and polls; the poll
// gives up after `spin` rounds (a launch argument; 0 gives up at once), and
// then no later barrier of the launch waits, so every wave finishes.  A
// workgroup that gave up sets the problem's status word, which the host reads
// with the truncation result and turns into an error before anything of the
// MPO is written.
static_assert(QMW_ROWS * QMW_MAXWG >= QPN, "every panel row needs a thread");
static_assert(2 * (QNB - 1) + 8 <= QMW_VALS && QMW_ROWS / 64 == 4, "partial layout");

// Per-wave sums of C values per lane through LDS: each wave writes its
// values value-major (stride 65 doubles, so a wave's write and the summing
// threads' reads spread over the banks), then thread (w, i) adds the 64
// entries of value i of wave w with four accumulators in a fixed order --
// one pass instead of C dependent shuffle chains.  red[w][i] <- the sum.
constexpr int QMW_LD = 65;
template <int C>
__device__ __forceinline__ void qmw_block_sum(const double (&vals)[C], double (*red)[QMW_VALS], double* big, int tid) {
  const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int i = 0; i < C; ++i) big[(wv * C + i) * QMW_LD + lane] = vals[i];
  __syncthreads();
  if (tid < 4 * C) {
    const int w = tid / C, i = tid - w * C;
    const double* p = big + (w * C + i) * QMW_LD;
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll
    for (int l = 0; l < 64; l += 4) {
      s0 += p[l];
      s1 += p[l + 1];
      s2 += p[l + 2];
      s3 += p[l + 3];
    }
    red[w][i] = (s0 + s1) + (s2 + s3);
  }
}

template <typename T>
__global__ __launch_bounds__(QMW_ROWS) void k_qr_panel(QrBatch qb, QrSyncBatch sb, int p0) {
  const int pi = blockIdx.y;
  if (pi >= qb.count) return;
  const QrProb P = qb.p[pi];
  if (p0 >= P.r) return;
  const int n = P.n, N = n - p0;
  const int nwg = (N + QMW_ROWS - 1) / QMW_ROWS;
  const int w = blockIdx.x;
  if (w >= nwg) return;
  const int nb = min(QNB, P.r - p0);
  const QrSyncProb S = sb.p[pi];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int rr = w * QMW_ROWS + tid;   // panel row (absolute row p0 + rr)
  const bool live = rr < N;
  const int rcl = min(rr, N - 1);
  cx<T>* M = (cx<T>*)P.M;
  cx<T>* tau = (cx<T>*)P.tau;
  cx<T>* Tf = (cx<T>*)P.Tf + (size_t)(p0 / QNB) * QNB * QNB;
  cx<double> a[QNB];
  {
    // all loads first (clamped addresses), then the masks and conversions
    cx<T> raw[QNB];
#pragma unroll
    for (int k = 0; k < QNB; ++k) raw[k] = M[(size_t)(p0 + min(k, nb - 1)) * n + p0 + rcl];
#pragma unroll
    for (int k = 0; k < QNB; ++k) {
      const double mk = (live && k < nb) ? 1.0 : 0.0;
      a[k] = cx<double>{mk * (double)raw[k].re, mk * (double)raw[k].im};
    }
  }
  __shared__ double red[QMW_ROWS / 64][QMW_VALS];
  __shared__ double big[QMW_ROWS / 64 * (2 * (QNB - 1) + 8) * QMW_LD];
  __shared__ double tot[QMW_VALS];
  __shared__ cx<double> Tl[QNB][QNB + 1];
  __shared__ int timed_out;
  if (tid == 0) timed_out = S.spin <= 0 ? 1 : 0;
  unsigned bar = 0;   // barriers passed in this launch (uniform)
  // block partials red[][0:C) -> this workgroup's slot, barrier, sum over
  // workgroups in order -> tot[0:C).  One release (thread 0's add; the
  // block barrier before it orders the other threads' stores) and one
  // acquire (thread 0's fence after the wait; the block barrier after it
  // orders the other threads' loads) per barrier.
  auto grid_sum = [&](int C) {
    __syncthreads();
    if (nwg == 1) {
      // a panel of at most QMW_ROWS rows: no other workgroup to meet, so no
      // counter, no agent-scope release/acquire and no round trip through
      // memory (the sum is the one the exchange would give: 0 + x)
      if (tid < C) tot[tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
      __syncthreads();
      return;
    }
    double* mine = S.part + ((size_t)(bar & 1) * QMW_MAXWG + w) * QMW_VALS;
    if (tid < C) mine[tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
    __syncthreads();
    ++bar;
    if (tid == 0) {
      __hip_atomic_fetch_add(S.cnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned target = S.base + bar * (unsigned)nwg;
      int it = 0;
      while (!timed_out &&
             (int)(__hip_atomic_load(S.cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
        __builtin_amdgcn_s_sleep(1);
        if (++it > S.spin) timed_out = 1;   // no later barrier of this launch waits either
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    if (tid < C) {
      const double* all = S.part + (size_t)((bar - 1) & 1) * QMW_MAXWG * QMW_VALS + tid;
      double v[QMW_MAXWG];
#pragma unroll
      for (int u = 0; u < QMW_MAXWG; ++u) v[u] = all[(size_t)min(u, nwg - 1) * QMW_VALS];
      double t = 0;
#pragma unroll
      for (int u = 0; u < QMW_MAXWG; ++u)
        if (u < nwg) t += v[u];
      tot[tid] = t;
    }
    __syncthreads();
  };

  double xn2 = 0, ar = 0, ai = 0;   // column j's tail norm and alpha, when carried over
  bool exact = true;                // sum column j's tail norm directly
  // The column loop is unrolled (a constant trip count, the body guarded by
  // the uniform j < nb), so every access to the register array a[] has a
  // constant index: a loop with a variable j would turn each of them into a
  // chain of selects over all QNB entries.
#pragma unroll
  for (int j = 0; j < QNB; ++j) {
    if (j < nb) {
      cx<double> xj{0.0, 0.0};
#pragma unroll
      for (int k = 0; k < QNB; ++k)
        if (k == j) xj = a[k];
      if (exact) {
        const double v1[3] = {rr > j ? xj.re * xj.re + xj.im * xj.im : 0.0, rr == j ? xj.re : 0.0,
                              rr == j ? xj.im : 0.0};
        qmw_block_sum<3>(v1, red, big, tid);
        grid_sum(3);
        xn2 = tot[0];
        ar = tot[1];
        ai = tot[2];
      }
      double tr = 0, ti = 0, scr = 0, sci = 0, beta = ar;
      if (xn2 > 0 || ai != 0) {
        const double nrm = sqrt(ar * ar + ai * ai + xn2);
        beta = (ar >= 0) ? -nrm : nrm;
        tr = (beta - ar) / beta;
        ti = -ai / beta;
        const double dr = ar - beta, di = ai, d2 = dr * dr + di * di;
        scr = dr / d2;
        sci = -di / d2;
      }
      const bool trivial = (tr == 0.0 && ti == 0.0);
      // this row of column j: beta on the diagonal, the scaled tail below
      cx<double> vj{0.0, 0.0};
      if (rr == j) {
        xj = cx<double>{beta, 0.0};
        vj = cx<double>{1.0, 0.0};
      } else if (rr > j) {
        if (!trivial) xj = cx<double>{xj.re * scr - xj.im * sci, xj.re * sci + xj.im * scr};
        vj = xj;
      }
#pragma unroll
      for (int k = 0; k < QNB; ++k)
        if (k == j) a[k] = xj;
      // w_k (slot k - 1, k > j), z_q (slot q, q < j), and column j + 1's
      // A, B, C and row-(j + 1) entries of a_{j+1} and v_j (slots 30..37)
      const int jn = j + 1;
      {
        constexpr int NV = 2 * (QNB - 1) + 8;
        double v2[NV];
        cx<double> an{0.0, 0.0};
#pragma unroll
        for (int sidx = 0; sidx < QNB - 1; ++sidx) {
          const bool isw = sidx >= j;
          const cx<double> ak = a[sidx + 1];
          const cx<double> aq = a[sidx];
          if (sidx + 1 == jn) an = ak;
          const cx<double> vq = (rr == sidx) ? cx<double>{1.0, 0.0} : (rr > sidx ? aq : cx<double>{0.0, 0.0});
          // w: conj(vj) a_k ; z: conj(vq) vj
          const cx<double> x = isw ? vj : vq, y = isw ? ak : vj;
          v2[2 * sidx] = x.re * y.re + x.im * y.im;
          v2[2 * sidx + 1] = x.re * y.im - x.im * y.re;
        }
        const bool below = rr > jn, at = rr == jn;
        v2[30] = below ? an.re * an.re + an.im * an.im : 0.0;
        v2[31] = below ? an.re * vj.re + an.im * vj.im : 0.0;   // conj(a) v
        v2[32] = below ? an.re * vj.im - an.im * vj.re : 0.0;
        v2[33] = below ? vj.re * vj.re + vj.im * vj.im : 0.0;
        v2[34] = at ? an.re : 0.0;
        v2[35] = at ? an.im : 0.0;
        v2[36] = at ? vj.re : 0.0;
        v2[37] = at ? vj.im : 0.0;
        qmw_block_sum<NV>(v2, red, big, tid);
      }
      grid_sum(2 * (QNB - 1) + 8);
      // a_k -= conj(tau) w_k v_j for k > j
      const double ctr = tr, cti = -ti;
#pragma unroll
      for (int k = 1; k < QNB; ++k) {
        if (k > j) {
          const double wr = tot[2 * (k - 1)], wi = tot[2 * (k - 1) + 1];
          const double fr = ctr * wr - cti * wi, fi = ctr * wi + cti * wr;
          a[k].re -= vj.re * fr - vj.im * fi;
          a[k].im -= vj.re * fi + vj.im * fr;
        }
      }
      // column j + 1's tail norm and alpha from the expansion, unless it may
      // have cancelled
      if (jn < nb) {
        const double wr = tot[2 * j], wi = tot[2 * j + 1];
        const double cr = ctr * wr - cti * wi, ci = ctr * wi + cti * wr;   // c = conj(tau) w_{j+1}
        const double A = tot[30], Br = tot[31], Bi = tot[32], Cv = tot[33];
        const double c2 = cr * cr + ci * ci;
        const double est = A - 2.0 * (cr * Br - ci * Bi) + c2 * Cv;
        const double scale = A + 2.0 * sqrt(c2 * (Br * Br + Bi * Bi)) + c2 * Cv;
        exact = !(est >= 0.1 * scale);
        xn2 = est;
        // alpha' = a_{j+1}[j+1] - c v_j[j+1]
        ar = tot[34] - (cr * tot[36] - ci * tot[37]);
        ai = tot[35] - (cr * tot[37] + ci * tot[36]);
      }
      // column j of T
      if (tid == 0) Tl[j][j] = cx<double>{tr, ti};
      if (tid < j) {
        double sr = 0, si = 0;
        for (int b = tid; b < j; ++b) {
          const cx<double> t = Tl[tid][b];
          const double zr = tot[2 * b], zi = tot[2 * b + 1];
          sr += t.re * zr - t.im * zi;
          si += t.re * zi + t.im * zr;
        }
        Tl[tid][j] = cx<double>{-(tr * sr - ti * si), -(tr * si + ti * sr)};
      }
      if (w == 0 && tid == 0) tau[p0 + j] = cx<T>{(T)tr, (T)ti};
      __syncthreads();
    }
  }
  if (live) {
#pragma unroll
    for (int k = 0; k < QNB; ++k)
      if (k < nb) M[(size_t)(p0 + k) * n + p0 + rr] = cx<T>{(T)a[k].re, (T)a[k].im};
  }
  if (w == 0 && tid < QNB * QNB) {
    const int ta = tid / QNB, tb = tid % QNB;
    const cx<double> t = (ta < nb && tb < nb && ta <= tb) ? Tl[ta][tb] : cx<double>{0, 0};
    Tf[tid] = cx<T>{(T)t.re, (T)t.im};
  }
  if (tid == 0) {
    if (timed_out) *S.fail = 1;
    // barriers not taken (norms carried over) still count, so the counter
    // ends at base + 2 nb per workgroup as the caller expects; every
    // workgroup has passed the last barrier here, so no wait is disturbed
    const unsigned rest = 2u * (unsigned)nb - bar;
    if (rest) __hip_atomic_fetch_add(S.cnt, rest, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <typename T>
void launch_qr_panel(const QrBatch& b, const QrSyncBatch& sy, int p0, int maxwg, hipStream_t s) {
  hipLaunchKernelGGL(k_qr_panel<T>, dim3(maxwg, b.count), dim3(QMW_ROWS), 0, s, b, sy, p0);
}
template <typename T>
void launch_qr_apply(const QrApplyBatch& b, int p0, int maxcols, hipStream_t s) {
  const int gx = (maxcols + QAT - 1) / QAT;
  int maxrows = 0;
  for (int p = 0; p < b.count; ++p)
    if (p0 < b.p[p].r && b.p[p].c0 < b.p[p].c1 && b.p[p].n - p0 > maxrows) maxrows = b.p[p].n - p0;
  if (gx < 1 || maxrows < 1) return;
  hipLaunchKernelGGL(k_qr_w1<T>, dim3(gx, (maxrows + QRC1 - 1) / QRC1, b.count), dim3(256), 0, s, b, p0);
  hipLaunchKernelGGL(k_qr_w2<T>, dim3(gx, b.count), dim3(256), 0, s, b, p0);
  hipLaunchKernelGGL(k_qr_upd<T>, dim3(gx, (maxrows + QRC2 - 1) / QRC2, b.count), dim3(256), 0, s, b, p0);
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
  template void launch_qr_panel<T>(const QrBatch&, const QrSyncBatch&, int, int, hipStream_t); \
  template void launch_qr_apply<T>(const QrApplyBatch&, int, int, hipStream_t);   \
  template void launch_lower_from_r<T>(const LowerBatch&, int, int, hipStream_t); \
  template void launch_build_y<T>(const VkBatch&, size_t, hipStream_t);           \
  template void launch_vh_rows<T>(const VkBatch&, size_t, hipStream_t);
QINST(float)
QINST(double)

}  // namespace mpo

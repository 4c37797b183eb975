// Internal types shared by the kernels and the host runtime of libmpo.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpo {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};

// Up to this many independent problems travel in one launch; their
// descriptors are passed by value as kernel arguments.
constexpr int MAXB = 32;
// Column-block width of the block one-sided Jacobi SVD (a block pair is a
// panel of 2*JB columns).
constexpr int JB = 16;
// Rows per workgroup of the Jacobi Gram and rotation kernels.
constexpr int GRC = 512;
constexpr int RRC = 256;   // default rotation row chunk (the launch passes its own)
// Panel rotation launch: every row on FP MFMA, or (mixed form) theta's rows
// on split-BF16 products and V's rows on FP32 MFMA in the same launch.
constexpr int ROT_FP = 0, ROT_MIXED = 1;

// ---------------------------------------------------------------- GEMM
// C[M x N] = C0 + A[M x K] * op(B), complex, row-major (C0 = 0 when null;
// C0 has C's leading dimension and must not alias A or B).
//   bmode 0: B is K x N row-major (ldb)
//   bmode 1: op(B) = conj(W)^T with W an N x K row-major matrix (ldb)
//   herm: the result is Hermitian; tiles of GEMM_TILE x GEMM_TILE entirely
//         below the diagonal are not computed (their entries are left as is)
constexpr int GEMM_TILE = 64;
struct GemmProb {
  const void* A;
  const void* B;
  void* C;
  int M, N, K;
  int lda, ldb, ldc;
  int bmode;
  int herm;
  const void* C0;
};
struct GemmBatch {
  GemmProb p[MAXB];
  int count;
};

// ---------------------------------------------------------------- gate
// theta0 (m x n row-major, m = 4 chil, n = 4 chir) -> theta_nolam (same) and
// M = conj(lam[a] * theta) in the same row-major positions, i.e. the column-
// major n x m matrix (lam theta)^dag; M may alias theta0.
struct GateProb {
  const void* theta0;
  void* theta_nolam;
  void* M;
  const double* lam;      // chil values (FP64)
  const double* gates;    // 64 doubles: g_out (32) then g_in (32), device
  int chil, chir;
  int has_out, has_in;
};
struct GateBatch {
  GateProb p[MAXB];
  int count;
};

// ---------------------------------------------------------------- Jacobi
struct JacState {
  int active;     // still sweeping
  int rot;        // block pairs rotated in the current sweep
  int sweeps;     // sweeps run
  int rot_total;  // block pairs rotated over all sweeps
  int epoch;      // sweeps launched (converged or not): the step stamp of step s
                  // of the current sweep is epoch * nblk + s + 1, so stamps
                  // grow without host arguments (a captured sweep replays as is)
};
struct JacProb {
  void* A;        // column-major, lda rows allocated, m used, ncol_pad columns
  void* V;        // column-major, ldv = ncol_pad rows, ncol_pad columns (NULL: values only)
  JacState* st;
  double* norms;  // ncol_pad column norms (output of the norm kernel)
  cx<double>* gpart;  // per pair, ngchunk partial 32x32 Gram matrices
  void* dmat;     // per pair, D = W - I (32x32, working precision)
  int* pflag;     // per pair, 1 if the panel is rotated in this step
  // Skipping of unchanged converged pairs: bmod[b] is the step stamp of the
  // last rotation of block b, pchk[bi * nblk + bj] the stamp at which the pair
  // was last found converged.  A pair with pchk > bmod of both blocks would
  // reproduce the same Gram matrix bit for bit and the same decision, so its
  // Gram and EVD are skipped.  Valid within one tolerance; k_jac_init clears it.
  int* bmod;
  int* pchk;
  double tol;     // off-diagonal tolerance |g_ij| <= tol sqrt(g_ii g_jj)
  int m, lda, ncol, ncol_pad, nblk, ngchunk;
};
// Round-robin pairing of N (even) indices: in step `step` (0 <= step < N - 1)
// pair t (0 <= t < N / 2) is (a, b), a < b; every index appears once per step
// and every pair once per N - 1 steps.
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

// Operand column of panel column c (0 <= c < 2 JB): block bi, then block bj.
__device__ __forceinline__ int panel_col(int bi, int bj, int c) { return c < JB ? bi * JB + c : bj * JB + c - JB; }

__device__ __forceinline__ bool pair_unchanged(const JacProb& P, int bi, int bj) {
  const int c = P.pchk[bi * P.nblk + bj];
  return c > 0 && c > P.bmod[bi] && c > P.bmod[bj];
}
struct JacBatch {
  JacProb p[MAXB];
  int count;
};

// Column ordering of the Jacobi operand before the first sweeps (second-QR
// route): the columns by decreasing norm, ties by index; the pair-skip
// bookkeeping is cleared since the blocks then hold other columns.
struct ColSortProb {
  const double* norms;  // ncol_pad column norms of the operand
  int* perm;            // out: perm[j] = the column that goes to position j
  const void* A;        // operand, column-major, lda x ncol_pad
  void* A2;             // out: the operand with its columns in that order
  int* pchk;
  int* bmod;
  int m, lda, ncol, ncol_pad, nblk;
  int on;               // 0: this problem is left as it is (both kernels skip it)
};
struct ColSortBatch {
  ColSortProb p[MAXB];
  int count;
};

// ---------------------------------------------------------------- QR
// Householder QR of M (n x m, column-major, leading dimension n) over its
// first r = min(n, m) columns, in panels of QNB columns: R on and above the
// diagonal, the reflector vectors v (unit first entry implied) below it,
// tau[j] per reflector and, per panel, the upper-triangular T of the compact
// WY form  H_p0 ... H_p0+nb-1 = I - V T V^dag.
constexpr int QNB = 16;
constexpr int QAT = 16;   // columns per workgroup of the reflector application
struct QrProb {
  void* M;
  void* tau;      // r entries
  void* Tf;       // ceil(r / QNB) panels x QNB x QNB, row-major per panel
  int n, m, r;
};
struct QrBatch {
  QrProb p[MAXB];
  int count;
};
// C (n rows, leading dimension ldc, columns [c0, c1)) <- (I - V op(T) V^dag) C
// for the panel starting at column p0 of M; op(T) = T^dag (Q^dag from the left,
// used for the trailing matrix) or T (Q from the left, used to form V).
// The product V^dag C is summed in two levels: k_qr_w1 writes one FP64
// partial per QRC1-row chunk (wpart: chunks x QNB x ldp), k_qr_w2 adds them in
// chunk order and multiplies by op(T) (w2: QNB x ldp), k_qr_upd subtracts V w2.
constexpr int QRC1 = 512;
constexpr int QRC2 = 256;
// Panel factorisation: the panel's rows are spread over up to
// QMW_MAXWG workgroups of QMW_ROWS threads (one row each); the workgroups of a
// problem exchange FP64 partial sums through `part` and meet at barriers on
// the counter `cnt`, which only ever grows (compared modulo 2^32): a launch
// starts at `base` and adds 2 nb per workgroup (at most two barriers per
// column; the ones not taken are added at the end).
constexpr int QMW_ROWS = 256;
constexpr int QMW_MAXWG = 16;
constexpr int QMW_VALS = 40;        // doubles per workgroup partial
struct QrSyncProb {
  unsigned* cnt;
  double* part;    // 2 (alternating by barrier) x QMW_MAXWG x QMW_VALS
  unsigned base;
  int spin;        // polls before a barrier gives up (0: give up at once)
  int* fail;       // set to 1 when a barrier gave up (the problem's status word)
};
struct QrSyncBatch {
  QrSyncProb p[MAXB];
};
struct QrApplyProb {
  const void* M;
  const void* Tf;
  void* C;
  void* wpart;    // cx<double>, ceil(n / QRC1) * QNB * ldp
  void* w2;       // cx<T>, QNB * ldp
  int n, r, ldc, c0, c1, ldp;   // columns of C index wpart / w2 directly (c1 <= ldp)
};
struct QrApplyBatch {
  QrApplyProb p[MAXB];
  int count;
  int conj_t;     // 1: T^dag, 0: T
};

// A[j * lda + i] = conj(R[j][i]) = conj(M[i * n + j]) for i >= j (i < m, j < r);
// zero above the diagonal and in the padding columns j in [r, rpad).
struct LowerProb {
  const void* M;
  void* A;
  int n, m, r, rpad, lda;
};
struct LowerBatch {
  LowerProb p[MAXB];
  int count;
};

struct VkProb {
  const void* W;        // column-major, ldw rows
  const int* perm;
  const double* s_sorted;
  void* Y;              // n x k column-major (ld n)
  void* right;          // k x n row-major
  double* lam;
  int n, r, k, ldw;
};
struct VkBatch {
  VkProb p[MAXB];
  int count;
};

// ---------------------------------------------------------------- truncation
struct TruncResult {
  int k;
  int nvals;
  double discarded;
  double total;
  double s0;
  int bad;        // non-finite singular value seen
  int qr_fail;    // a QR panel barrier gave up: the factorisation is invalid
};
struct TruncProb {
  const double* norms;   // ncol_pad column norms
  double* s_sorted;      // descending
  int* perm;             // column index of each sorted value
  TruncResult* res;
  double cutoff;
  int ncol, ncol_pad;
  int nval;              // number of singular values: min(rows, columns)
  int chi_max, mode;
};
struct TruncBatch {
  TruncProb p[MAXB];
  int count;
};

}  // namespace mpo

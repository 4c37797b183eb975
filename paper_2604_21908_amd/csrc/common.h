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

// ---------------------------------------------------------------- GEMM
// C[M x N] = A[M x K] * op(B), complex, row-major.
//   bmode 0: B is K x N row-major (ldb)
//   bmode 1: op(B) = conj(W)^T with W an N x K row-major matrix (ldb)
struct GemmProb {
  const void* A;
  const void* B;
  void* C;
  int M, N, K;
  int lda, ldb, ldc;
  int bmode;
};
struct GemmBatch {
  GemmProb p[MAXB];
  int count;
};

// ---------------------------------------------------------------- gate
// theta0 (m x n row-major, m = 4 chil, n = 4 chir) -> theta_nolam (same) and
// A = lam[a] * theta, column-major with leading dimension lda.
struct GateProb {
  const void* theta0;
  void* theta_nolam;
  void* A;
  const double* lam;      // chil values (FP64)
  const double* gates;    // 64 doubles: g_out (32) then g_in (32), device
  int chil, chir, lda;
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
  int pad;
};
struct JacProb {
  void* A;        // column-major, lda rows allocated, m used, ncol_pad columns
  void* V;        // column-major, ldv = ncol_pad rows, ncol_pad columns (NULL: values only)
  JacState* st;
  double* norms;  // ncol_pad column norms (output of the norm kernel)
  double tol;     // off-diagonal tolerance |g_ij| <= tol sqrt(g_ii g_jj)
  int m, lda, ncol, ncol_pad, nblk;
};
struct JacBatch {
  JacProb p[MAXB];
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
  int pad;
};
struct TruncProb {
  const double* norms;   // ncol_pad column norms
  double* s_sorted;      // descending
  int* perm;             // column index of each sorted value
  TruncResult* res;
  int ncol, ncol_pad;
  int nval;              // number of singular values: min(rows, columns)
};
struct TruncBatch {
  TruncProb p[MAXB];
  int count;
  int chi_max;
  int mode;
  double cutoff;
};

// ---------------------------------------------------------------- write-back
struct WbProb {
  const void* V;       // column-major, ldv rows
  const int* perm;
  const double* s_sorted;
  void* right;         // new B_{i+1}: k x ncol row-major
  double* lam;         // new lambda_i: k values
  int ldv, ncol, k;
};
struct WbBatch {
  WbProb p[MAXB];
  int count;
};

}  // namespace mpo

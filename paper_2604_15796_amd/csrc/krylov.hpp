// Batched restarted GMRES kernels (the Krylov solver of Sec. IV-A), one
// independent Arnoldi process per right-hand side, all advanced in lockstep.
// Inner products, norms, the Hessenberg matrix, Givens rotations and the
// solution accumulator are FP64; the basis may be complex64 or complex128.
#pragma once

#include "internal.hpp"

namespace fwi {

// Device state of one batched GMRES cycle.
template <typename T>
struct KrylovState {
  int B = 0, JM = 0;   // right-hand sides, basis capacity (restart length)
  long n = 0;          // unknowns per RHS
  int nblk = 0, chunk = 0;
  cplx<T>* V = nullptr;        // [JM+1][B][n]
  c128* H = nullptr;           // [B][JM+1][JM]
  double* cs = nullptr;        // [B][JM]
  c128* sn = nullptr;          // [B][JM]
  c128* gv = nullptr;          // [B][JM+1]
  c128* y = nullptr;           // [B][JM] correction x += sum_i y_i V_i (stored V_i; |r| and scales folded in)
  c128* dotp = nullptr;        // [B][parts][JM+1]: nblk parts (k_dots) or one per inverse-row-pass workgroup
  c128* hcoef = nullptr;       // [B][JM+1] Gram-Schmidt coefficients of the current step
  double* nrmp = nullptr;      // [B][nblk]
  double* rnorm = nullptr;     // [B] residual norm at cycle start
  double* bnorm = nullptr;     // [B]
  double* target = nullptr;    // [B] relative stopping target of the cycle
  double* rscale = nullptr;    // [B] 1/rnorm
  cplx<T>* vscale = nullptr;   // [JM+1][B] basis vector i of RHS b = vscale * stored V_i
  int* active = nullptr;       // [B]
  int* ncol = nullptr;         // [B]
  int* iters = nullptr;        // [B] accumulated iterations
  int* counters = nullptr;     // [0] active count, [1] unconverged
  double* maxrel = nullptr;    // [1] max relative residual at cycle start
  long vstride() const { return (long)B * n; }
};

int krylov_nblk(long n);

// V_0 was written by the first pass of the first cycle (b) or by the residual
// epilogue of the operator (later cycles) together with one |r|^2 partial per
// grid row; fold those into nrmp.
template <typename T>
void krylov_rows_norm(const KrylovState<T>& s, const double* rowpart, int rows, hipStream_t st);
// Norms, activity, stopping targets and the scale of V_0 (1 / |r|).
template <typename T>
void krylov_cycle_init(const KrylovState<T>& s, int first, double rtol, double inner_rtol, hipStream_t st);
// Arnoldi step j after the matvec w = A v_j stored into V_{j+1}:
// inner products of w with V_0..V_j in nblk parts per RHS (used when the
// operator's last pass could not produce them);
template <typename T>
void krylov_dots(const KrylovState<T>& s, int j, hipStream_t st);
// column j of H from ndot parts per RHS and the Gram-Schmidt coefficients
// (hcoef) that the first pass of the next matvec applies to w (see OrthIn);
template <typename T>
void krylov_hsum(const KrylovState<T>& s, int j, int ndot, hipStream_t st);
// after that pass: the norm of the orthogonalised vector from its per-row
// sums (rows per RHS), Givens rotations, convergence, scale of V_{j+1} and
// the active count.
template <typename T>
void krylov_givens(const KrylovState<T>& s, int j, const double* rowpart, int rows, hipStream_t st);
// Back-substitution: y from the rotated Hessenberg system, scaled so that
// the correction is sum_{i < ncol} y_i V_i over the stored basis vectors.
template <typename T>
void krylov_backsolve(const KrylovState<T>& s, hipStream_t st);
// x += sum_{i < ncol} y_i V_i; first: x is written, not read (x_0 = 0).
template <typename T>
void krylov_xupdate(const KrylovState<T>& s, c128* x, int first, hipStream_t st);
// Both of the above.
template <typename T>
void krylov_finish_cycle(const KrylovState<T>& s, c128* x, int first, hipStream_t st);
template <typename T>
void krylov_reset_iters(const KrylovState<T>& s, hipStream_t st);

void launch_fill_zero_c128(long count, c128* p, hipStream_t st);
// st[0] = max(st[0], max_b iters[b]), st[1] += sum_b iters[b]
void launch_iter_stats(int B, const int* iters, unsigned long long* st, hipStream_t s);
void launch_zero_u64(int count, unsigned long long* p, hipStream_t s);
void launch_copy_c128(long count, const c128* in, c128* out, hipStream_t st);

}  // namespace fwi

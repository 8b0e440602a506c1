// Launchers of the data-space / model-space kernels (see kern_data.hip).
#pragma once

#include "internal.hpp"

namespace fwi {

// C[l][i][j] = coef[l] sum_n A[l][i][n] w[n] Bm[l][j][n]; part: [nks][nf][ni][nj] scratch
void launch_gemm_nt(int nf, const c128* A, long a_ls, int ni, const c128* w, const c128* Bm, long b_ls, int nj, long n,
                    const c128* coef, c128* part, int nks, c128* C, hipStream_t st);
// S[l][i][n] = sum_j conj(M[l][i][j]) P[l][j][n]
void launch_gemm_cn(int nf, const c128* M, int ni, int nj, const c128* P, long p_ls, long n, c128* S, long s_ls,
                    hipStream_t st);
// r = data - dobs (dobs may be null), misfit = 1/2 |r|^2
void launch_residual(long count, const c128* data, const c128* dobs, c128* r, double* misfit, hipStream_t st);
// acc (+)= sum_l conj(k2_l) sum_i conj(p_li lam_li) over the nf x ni fields given; part: [nseg][n]
void launch_gradient_accum(long n, int nf, int ni, const c128* p, const c128* lam, const c128* k2, c128* part,
                           int nseg, int first, c128* acc, hipStream_t st);
// g = dV acc and the chain rule to c, alpha (each output may be null)
void launch_grad_chain(long n, const c128* acc, double dV, c128 ik0r, const double* c, const double* alpha, c128* g,
                       double* gc, double* ga, hipStream_t st);
void launch_tv_grad(const Geo& g, const c128* m, c128* out, hipStream_t st);
void launch_tv_gradT(const Geo& g, const c128* a, double alpha, double beta, c128* out, hipStream_t st);
int launch_tv_shrink_dual(const Geo& g, const c128* gm, double tau, double dual, c128* gout, c128* u, double* tvp,
                          hipStream_t st);
void launch_lincomb(long n, double a, const c128* x, double b, const c128* y, double c, const c128* z, c128* out,
                    hipStream_t st);
int dot_blocks(long n);
void launch_dot_re(long n, const c128* x, const c128* y, double* part, double* out, hipStream_t st);
void launch_sum(int nb, const double* part, double* out, hipStream_t st);
void launch_cg_step1(long n, const double* sc, c128* x, c128* r, const c128* p, const c128* Ap, hipStream_t st);
void launch_cg_step2(long n, const double* sc, const c128* r, c128* p, hipStream_t st);
void launch_copy_scalar(const double* in, double* out, hipStream_t st);
void launch_conj_c128(long count, const c128* in, c128* out, hipStream_t st);
// J^H b in one pass over the receiver fields: S = conj(M) P as in
// launch_gemm_cn, reduced on the fly with the transmit fields T into
// conj(k2) conj(T S) partials part [nf * ceil(ni / 64)][n]; launch_grad_sum
// adds such partials (or those of launch_gradient_accum) in a fixed order.
int gemm_cn_grad_segments(int nf, int ni);
void launch_gemm_cn_grad(int nf, const c128* M, int ni, int nj, const c128* P, long p_ls, long n, const c128* T,
                         long t_ls, const c128* k2, c128* part, hipStream_t st);
void launch_grad_sum(long n, const c128* part, int nseg, int first, c128* acc, hipStream_t st);
// coarse inversion mesh (factor r) <-> forward mesh g: piecewise-constant
// prolongation and its adjoint
void launch_prolong(const Geo& g, int r, const c128* mc, c128* mf, hipStream_t st);
void launch_restrict(const Geo& g, int r, const c128* gf, c128* gcv, hipStream_t st);
void launch_fill_rfreq(int B, int per, int l0, int* rf, hipStream_t st);

}  // namespace fwi

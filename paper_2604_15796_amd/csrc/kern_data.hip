// Data-space and model-space kernels of the gradient and ADMM path:
//  * receiver sampling / forward Jacobian product (Eq. 4, Eq. 16):
//      C[l][i][j] = coef_l sum_n A[l][i][n] w[n] Bm[l][j][n]
//  * residual and misfit (data term of Eq. 7)
//  * adjoint sources / adjoint-field contraction (Eq. 17):
//      S[l][i][n] = sum_j conj(M[l][i][j]) P[l][j][n]
//  * gradient reduction g_n = dV sum_l conj(k_l^2) sum_i conj(p_li[n] lam_li[n])
//    and the chain rule to c and alpha
//  * TV operators, shrinkage and dual update (Eq. 13-14), CG vector updates.
// All accumulations are FP64 with fixed-order two-stage reductions.
#include "data.hpp"

namespace fwi {

constexpr double PI = 3.14159265358979323846;

// ------------------------------------------------- FP64 matrix-core tiles ---
// v_mfma_f64_16x16x4f64: D (16 x 16) += A (16 x 4) B (4 x 16), one value per
// lane and operand: A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k, and
// D[i][j] in lane j + 16 (i % 4), element i / 4 of the lane's four doubles.
typedef double v4d __attribute__((ext_vector_type(4)));

// Complex 16 x 16 tile (cr, ci) += A B from this lane's complex operands, as
// four real products.
__device__ __forceinline__ void cmfma(c128 a, c128 b, v4d& cr, v4d& ci) {
  cr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, cr, 0, 0, 0);
  cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, cr, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, ci, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, ci, 0, 0, 0);
}

// ------------------------------------------------------------- gemm (NT) ---
// 64 x 64 output tile per block of 4 waves: wave w owns rows 16w .. 16w+15 as
// four 16 x 16 complex tiles on the FP64 matrix cores; every A and Bm element
// of a split is read from HBM once per output tile and staged through LDS.
constexpr int GT = 64;  // output tile
constexpr int GK = 16;  // k step

// part[ks][l][i][j] = sum over the split's k range of A[l][i][k] w[k] Bm[l][j][k]
__global__ void __launch_bounds__(256) k_gemm_nt(const c128* __restrict__ A, long a_ls, int ni,
                                                 const c128* __restrict__ w, const c128* __restrict__ Bm, long b_ls,
                                                 int nj, long n, long kchunk, c128* __restrict__ part, int nf) {
  __shared__ c128 sa[GT][GK + 1];
  __shared__ c128 sb[GT][GK + 1];
  const int ks = blockIdx.x;
  const int tj_n = (nj + GT - 1) / GT;
  const int ti = blockIdx.y / tj_n, tj = blockIdx.y % tj_n;
  const int l = blockIdx.z;
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  const c128* Al = A + l * a_ls;
  const c128* Bl = Bm + l * b_ls;
  v4d cr[4], ci[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    cr[b] = v4d{0.0, 0.0, 0.0, 0.0};
    ci[b] = v4d{0.0, 0.0, 0.0, 0.0};
  }
  const long k0 = ks * kchunk;
  const long k1 = min(n, k0 + kchunk);
  // 64 x 16 tiles of A (rows ti*64 ..) and Bm (rows tj*64 ..), k in [kb, kb+16);
  // the next tile is loaded into registers while the current one is used
  // (raw loads only: the weight is applied at the LDS store, so no load is
  // waited for before the current tile's products)
  // Loads use clamped indices and are masked at the LDS store, so nothing
  // waits for them before the current tile's products.
  constexpr int Q = GT * GK / 256;
  c128 ra[Q], rb[Q], rw[Q];
  bool va[Q], vb[Q];
  auto fetch = [&](long kb) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = t + q * 256;
      const int r = e / GK, c = e % GK;
      const long k = kb + c;
      const int ia = ti * GT + r, jb = tj * GT + r;
      va[q] = k < k1 && ia < ni;
      vb[q] = k < k1 && jb < nj;
      const long kc = k < k1 ? k : k1 - 1;
      ra[q] = Al[(long)(ia < ni ? ia : ni - 1) * n + kc];
      rb[q] = Bl[(long)(jb < nj ? jb : nj - 1) * n + kc];
      rw[q] = w ? w[kc] : mk(1.0, 0.0);
    }
  };
  if (k0 < k1) fetch(k0);
  for (long kb = k0; kb < k1; kb += GK) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = t + q * 256;
      sa[e / GK][e % GK] = va[q] ? ra[q] * rw[q] : mk(0.0, 0.0);
      sb[e / GK][e % GK] = vb[q] ? rb[q] : mk(0.0, 0.0);
    }
    __syncthreads();
    if (kb + GK < k1) fetch(kb + GK);
#pragma unroll
    for (int c = 0; c < GK; c += 4) {
      // A[i][k] = sa[16 wv + i][c + k], B[k][j] = sb[16 b + j][c + k]
      const c128 av = sa[16 * wv + (lane & 15)][c + (lane >> 4)];
#pragma unroll
      for (int b = 0; b < 4; ++b) cmfma(av, sb[16 * b + (lane & 15)][c + (lane >> 4)], cr[b], ci[b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = ti * GT + 16 * wv + (lane >> 4) + 4 * v, j = tj * GT + 16 * b + (lane & 15);
      if (i < ni && j < nj) part[(((long)ks * nf + l) * ni + i) * nj + j] = mk(cr[b][v], ci[b][v]);
    }
}

// Sum of the split-K partials part[nks][tot] in a fixed order: a workgroup
// takes 64 consecutive outputs, wave w sums the splits w, w + 16, ... (one
// coalesced row of 64 per split), then the 16 wave sums are added in wave
// order.
__global__ void __launch_bounds__(1024) k_gemm_nt_final(const c128* __restrict__ part, int nks, int nf, int ni,
                                                        int nj, const c128* __restrict__ coef, c128* __restrict__ C) {
  __shared__ c128 red[16][64];
  const long tot = (long)nf * ni * nj;
  const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
  const long idx = (long)blockIdx.x * 64 + lane;
  c128 s = mk(0.0, 0.0);
  if (idx < tot)
    for (int k = w; k < nks; k += 16) s = s + part[(long)k * tot + idx];
  red[w][lane] = s;
  __syncthreads();
  if (w == 0 && idx < tot) {
    c128 t = red[0][lane];
#pragma unroll
    for (int q = 1; q < 16; ++q) t = t + red[q][lane];
    C[idx] = coef[(int)(idx / ((long)ni * nj))] * t;
  }
}

// ------------------------------------------------------------- gemm (NN) ---
// S[l][i][n] = sum_j conj(M[l][i][j]) P[l][j][n]: 64 (i) x 64 (n) output tile
// per block (wave w: rows 16w .. 16w+15, four 16 x 16 complex matrix-core
// tiles), j in steps of 16 through LDS; each P element is read from HBM once
// per 64 rows of S.
constexpr int CT = 64;  // output tile (rows of S, points n)
constexpr int CK = 16;  // j step

// GRAD: instead of storing S, the epilogue forms conj(k2[l]) conj(T[l][i][n] S[l][i][n])
// and sums it over the tile's 64 rows i in a fixed order (lane, then lanes
// 16 and 32 apart, then the four waves), one partial per (l, row tile, n) in
// part [nf][row tiles][n]: J^H b without storing the adjoint-like fields.
template <bool GRAD>
__global__ void __launch_bounds__(256) k_gemm_cn(const c128* __restrict__ M, int ni, int nj,
                                                 const c128* __restrict__ P, long p_ls, long n,
                                                 c128* __restrict__ S, long s_ls, const c128* __restrict__ T,
                                                 long t_ls, const c128* __restrict__ k2,
                                                 c128* __restrict__ part) {
  __shared__ c128 sm[CT][CK + 1];   // conj(M) tile [i][j]
  __shared__ c128 sp[CK][CT + 1];   // P tile [j][n]
  const int l = blockIdx.z;
  const int i0 = blockIdx.y * CT;
  const long n0 = (long)blockIdx.x * CT;
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  const c128* Ml = M + (long)l * ni * nj;
  const c128* Pl = P + l * p_ls;
  v4d cr[4], ci[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    cr[b] = v4d{0.0, 0.0, 0.0, 0.0};
    ci[b] = v4d{0.0, 0.0, 0.0, 0.0};
  }
  // M tile (row-major [i][j]) and P tile (n fastest, coalesced); the next pair
  // is loaded into registers while the current one is used
  // (clamped loads, masked at the LDS store: nothing waits for them early)
  constexpr int Q = CT * CK / 256;
  c128 rm[Q], rp[Q];
  bool vm[Q], vp[Q];
  auto fetch = [&](int jb) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = t + q * 256;
      {
        const int r = e / CK, c = e % CK;
        const int i = i0 + r, j = jb + c;
        vm[q] = i < ni && j < nj;
        rm[q] = Ml[(long)(i < ni ? i : ni - 1) * nj + (j < nj ? j : nj - 1)];
      }
      {
        const int r = e / CT, c = e % CT;
        const int j = jb + r;
        const long nn = n0 + c;
        vp[q] = j < nj && nn < n;
        rp[q] = Pl[(long)(j < nj ? j : nj - 1) * n + (nn < n ? nn : n - 1)];
      }
    }
  };
  fetch(0);
  for (int jb = 0; jb < nj; jb += CK) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = t + q * 256;
      sm[e / CK][e % CK] = vm[q] ? conj(rm[q]) : mk(0.0, 0.0);
      sp[e / CT][e % CT] = vp[q] ? rp[q] : mk(0.0, 0.0);
    }
    __syncthreads();
    if (jb + CK < nj) fetch(jb + CK);
#pragma unroll
    for (int c = 0; c < CK; c += 4) {
      // A[i][k] = sm[16 wv + i][c + k], B[k][j] = sp[c + k][16 b + j]
      const c128 mv = sm[16 * wv + (lane & 15)][c + (lane >> 4)];
#pragma unroll
      for (int b = 0; b < 4; ++b) cmfma(mv, sp[c + (lane >> 4)][16 * b + (lane & 15)], cr[b], ci[b]);
    }
    __syncthreads();
  }
  if constexpr (!GRAD) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + 16 * wv + (lane >> 4) + 4 * v;
      if (i >= ni) continue;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const long nn = n0 + 16 * b + (lane & 15);
        if (nn < n) S[l * s_ls + (long)i * n + nn] = mk(cr[b][v], ci[b][v]);
      }
    }
  } else {
    __shared__ c128 sred[4][CT];
    const c128 kc = conj(k2[l]);
    const c128* Tl = T + l * t_ls;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const long nn = n0 + 16 * b + (lane & 15);
      c128 acc = mk(0.0, 0.0);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + 16 * wv + (lane >> 4) + 4 * v;
        if (i < ni && nn < n) acc = acc + kc * conj(Tl[(long)i * n + nn] * mk(cr[b][v], ci[b][v]));
      }
      double ax = acc.x, ay = acc.y;
      ax += __shfl_xor(ax, 16, 64);
      ay += __shfl_xor(ay, 16, 64);
      ax += __shfl_xor(ax, 32, 64);
      ay += __shfl_xor(ay, 32, 64);
      if (lane < 16) sred[wv][16 * b + lane] = mk(ax, ay);
    }
    __syncthreads();
    if (t < CT && n0 + t < n) {
      const c128 s = ((sred[0][t] + sred[1][t]) + sred[2][t]) + sred[3][t];
      part[((long)l * gridDim.y + blockIdx.y) * n + n0 + t] = s;
    }
  }
}

// ------------------------------------------------------------- residual ---
__global__ void __launch_bounds__(1024) k_residual(long count, const c128* __restrict__ data,
                                                   const c128* __restrict__ dobs, c128* __restrict__ r,
                                                   double* __restrict__ misfit) {
  __shared__ double red[16];
  double acc = 0.0;
  for (long i = threadIdx.x; i < count; i += 1024) {
    const c128 v = dobs ? data[i] - dobs[i] : data[i];
    r[i] = v;
    acc += norm2(v);
  }
  const double s = block_sum<1024>(acc, red);
  if (threadIdx.x == 0) misfit[0] = 0.5 * s;
}

// ------------------------------------------------------------- gradient ---
// part[seg][n] = sum over the segment's (l, i) of conj(k_l^2) conj(p_li[n] lam_li[n])
__global__ void __launch_bounds__(256) k_grad_partial(const c128* __restrict__ p, const c128* __restrict__ lam,
                                                      long n, int nf, int ni, const c128* __restrict__ k2,
                                                      int nseg, c128* __restrict__ part) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const int seg = blockIdx.y;
  const long tot = (long)nf * ni;
  const long s0 = tot * seg / nseg, s1 = tot * (seg + 1) / nseg;
  c128 acc = mk(0.0, 0.0);
  for (long li = s0; li < s1; ++li) {
    const int l = (int)(li / ni);
    const c128 a = p[li * n + e], b = lam[li * n + e];
    const c128 prod = a * b;
    acc = acc + conj(k2[l]) * conj(prod);
  }
  part[(long)seg * n + e] = acc;
}

// acc (+)= sum_seg part  (fixed order)
__global__ void k_grad_accum(const c128* __restrict__ part, int nseg, long n, int first, c128* __restrict__ acc) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  c128 s = first ? mk(0.0, 0.0) : acc[e];
  for (int k = 0; k < nseg; ++k) s = s + part[(long)k * n + e];
  acc[e] = s;
}

// g = dV acc; optional chain rule d phi/dc = Re(conj(g) dm/dc), d phi/dalpha = Re(conj(g) dm/dalpha)
__global__ void k_grad_chain(const c128* __restrict__ acc, long n, double dV, c128 ik0r,
                             const double* __restrict__ c, const double* __restrict__ alpha,
                             c128* __restrict__ g, double* __restrict__ gc, double* __restrict__ ga) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const c128 s = dV * acc[e];
  if (g) g[e] = s;
  if (gc || ga) {
    const double cc = c[e], a = alpha ? alpha[e] : 0.0;
    // m = kappa rho / (kappa_0 rho_0) - 1 (ik0r = 1 / (kappa_0 rho_0)):
    // dm/dc = (-2/c^3 - i alpha/(pi c^2)) ik0r, dm/dalpha = (-2 alpha/(2 pi)^2 + i/(pi c)) ik0r
    const c128 dmc = mk(-2.0 / (cc * cc * cc), -a / (PI * cc * cc)) * ik0r;
    const c128 dma = mk(-2.0 * a / (4.0 * PI * PI), 1.0 / (PI * cc)) * ik0r;
    if (gc) gc[e] = s.x * dmc.x + s.y * dmc.y;
    if (ga) ga[e] = s.x * dma.x + s.y * dma.y;
  }
}

// ------------------------------------------------------------------- TV ---
struct TvGeo {
  int dim, nx, ny, nz;
};
__device__ __forceinline__ void tv_coords(const TvGeo& g, long i, int& ix, int& iy, int& iz) {
  ix = (int)(i % g.nx);
  iy = (int)((i / g.nx) % g.ny);
  iz = (int)(i / ((long)g.nx * g.ny));
}
// component q: 0 = x, 1 = y (3D) or z (2D), 2 = z (3D)
__device__ __forceinline__ void tv_axis(const TvGeo& g, int q, long& step, int& N, int ix, int iy, int iz, int& pos) {
  if (q == 0) {
    step = 1;
    N = g.nx;
    pos = ix;
  } else if (g.dim == 3 && q == 1) {
    step = g.nx;
    N = g.ny;
    pos = iy;
  } else {
    step = (long)g.nx * g.ny;
    N = g.nz;
    pos = iz;
  }
}

// out[q][i] = m[i + e_q] - m[i] (0 at the last index)
__global__ void k_tv_grad(TvGeo g, const c128* __restrict__ m, c128* __restrict__ out) {
  const long n = (long)g.nx * g.ny * g.nz;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int ix, iy, iz;
  tv_coords(g, i, ix, iy, iz);
  for (int q = 0; q < g.dim; ++q) {
    long st;
    int N, pos;
    tv_axis(g, q, st, N, ix, iy, iz, pos);
    out[(long)q * n + i] = pos < N - 1 ? m[i + st] - m[i] : mk(0.0, 0.0);
  }
}

// out[i] = sum_q (a_q[i - e_q] [pos >= 1] - a_q[i] [pos <= N-2]);  out = beta*out + alpha*that
__global__ void k_tv_gradT(TvGeo g, const c128* __restrict__ a, double alpha, double beta, c128* __restrict__ out) {
  const long n = (long)g.nx * g.ny * g.nz;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int ix, iy, iz;
  tv_coords(g, i, ix, iy, iz);
  c128 s = mk(0.0, 0.0);
  for (int q = 0; q < g.dim; ++q) {
    long st;
    int N, pos;
    tv_axis(g, q, st, N, ix, iy, iz, pos);
    if (pos >= 1) s = s + a[(long)q * n + i - st];
    if (pos <= N - 2) s = s - a[(long)q * n + i];
  }
  const c128 o = beta == 0.0 ? mk(0.0, 0.0) : beta * out[i];
  out[i] = o + alpha * s;
}

// g = shrink_tau(grad m - u); u += dual (g - grad m); tvp[block] = sum_n |grad m|_2
__global__ void __launch_bounds__(256) k_tv_shrink_dual(TvGeo gg, const c128* __restrict__ gm, double tau,
                                                        double dual, c128* __restrict__ g, c128* __restrict__ u,
                                                        double* __restrict__ tvp) {
  __shared__ double red[4];
  const long n = (long)gg.nx * gg.ny * gg.nz;
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  double tvl = 0.0;
  if (i < n) {
    c128 a[3];
    double nr = 0.0, ng = 0.0;
    for (int q = 0; q < gg.dim; ++q) {
      const c128 d = gm[(long)q * n + i];
      a[q] = d - u[(long)q * n + i];
      nr += norm2(a[q]);
      ng += norm2(d);
    }
    nr = sqrt(nr);
    tvl = sqrt(ng);
    const double fac = nr > 0.0 ? fmax(1.0 - tau / nr, 0.0) : 0.0;
    for (int q = 0; q < gg.dim; ++q) {
      const c128 gn = fac * a[q];
      g[(long)q * n + i] = gn;
      u[(long)q * n + i] = u[(long)q * n + i] + dual * (gn - gm[(long)q * n + i]);
    }
  }
  const double s = block_sum<256>(tvl, red);
  if (threadIdx.x == 0) tvp[blockIdx.x] = s;
}

// ------------------------------------------------------------- vectors ---
// out = a*x + b*y (+ c*z), real coefficients; x, y, z may alias out
__global__ void k_lincomb(long n, double a, const c128* x, double b, const c128* y, double c, const c128* z,
                          c128* out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  c128 v = a * x[i];
  if (y) v = v + b * y[i];
  if (z) v = v + c * z[i];
  out[i] = v;
}

// partial sums of Re <x, y> (x == y gives |x|^2)
__global__ void __launch_bounds__(256) k_dot_re_partial(long n, const c128* __restrict__ x, const c128* __restrict__ y,
                                                        double* __restrict__ part) {
  __shared__ double red[4];
  double acc = 0.0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    const c128 a = x[i], b = y[i];
    acc += a.x * b.x + a.y * b.y;
  }
  const double s = block_sum<256>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}
__global__ void k_sum_partial(int nb, const double* __restrict__ part, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < nb; ++k) s += part[k];
    out[0] = s;
  }
}

// CG scalars on device: sc[0] = rs, sc[1] = pAp, sc[2] = rs_new
// x += (rs/pAp) p ; r -= (rs/pAp) Ap
__global__ void k_cg_step1(long n, const double* __restrict__ sc, c128* __restrict__ x, c128* __restrict__ r,
                           const c128* __restrict__ p, const c128* __restrict__ Ap) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double rs = sc[0], pap = sc[1];
  const double al = (rs > 0.0 && pap != 0.0) ? rs / pap : 0.0;
  x[i] = x[i] + al * p[i];
  r[i] = r[i] - al * Ap[i];
}
// p = r + (rs_new/rs) p
__global__ void k_cg_step2(long n, const double* __restrict__ sc, const c128* __restrict__ r, c128* __restrict__ p) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double rs = sc[0], rsn = sc[2];
  const double be = rs > 0.0 ? rsn / rs : 0.0;
  p[i] = r[i] + be * p[i];
}
__global__ void k_copy_scalar(const double* __restrict__ in, double* __restrict__ out) {
  if (threadIdx.x == 0) out[0] = in[0];
}

// ------------------------------------------------------------- launchers ---
void launch_gemm_nt(int nf, const c128* A, long a_ls, int ni, const c128* w, const c128* Bm, long b_ls, int nj, long n,
                    const c128* coef, c128* part, int nks, c128* C, hipStream_t st) {
  long kchunk = (n + nks - 1) / nks;
  kchunk = (kchunk + GK - 1) / GK * GK;
  const int tiles = ((ni + GT - 1) / GT) * ((nj + GT - 1) / GT);
  hipLaunchKernelGGL(k_gemm_nt, dim3(nks, tiles, nf), dim3(256), 0, st, A, a_ls, ni, w, Bm, b_ls, nj, n, kchunk, part,
                     nf);
  FWI_LAUNCH_CHECK();
  const long tot = (long)nf * ni * nj;
  hipLaunchKernelGGL(k_gemm_nt_final, dim3((unsigned)((tot + 63) / 64)), dim3(1024), 0, st, part, nks, nf, ni, nj,
                     coef, C);
  FWI_LAUNCH_CHECK();
}

void launch_gemm_cn(int nf, const c128* M, int ni, int nj, const c128* P, long p_ls, long n, c128* S, long s_ls,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_gemm_cn<false>, dim3((unsigned)((n + CT - 1) / CT), (ni + CT - 1) / CT, nf), dim3(256), 0, st,
                     M, ni, nj, P, p_ls, n, S, s_ls, nullptr, 0L, nullptr, nullptr);
  FWI_LAUNCH_CHECK();
}
int gemm_cn_grad_segments(int nf, int ni) { return nf * ((ni + CT - 1) / CT); }
void launch_gemm_cn_grad(int nf, const c128* M, int ni, int nj, const c128* P, long p_ls, long n, const c128* T,
                         long t_ls, const c128* k2, c128* part, hipStream_t st) {
  hipLaunchKernelGGL(k_gemm_cn<true>, dim3((unsigned)((n + CT - 1) / CT), (ni + CT - 1) / CT, nf), dim3(256), 0, st,
                     M, ni, nj, P, p_ls, n, nullptr, 0L, T, t_ls, k2, part);
  FWI_LAUNCH_CHECK();
}
void launch_grad_sum(long n, const c128* part, int nseg, int first, c128* acc, hipStream_t st) {
  hipLaunchKernelGGL(k_grad_accum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, part, nseg, n, first, acc);
  FWI_LAUNCH_CHECK();
}

void launch_residual(long count, const c128* data, const c128* dobs, c128* r, double* misfit, hipStream_t st) {
  hipLaunchKernelGGL(k_residual, dim3(1), dim3(1024), 0, st, count, data, dobs, r, misfit);
  FWI_LAUNCH_CHECK();
}

void launch_gradient_accum(long n, int nf, int ni, const c128* p, const c128* lam, const c128* k2, c128* part,
                           int nseg, int first, c128* acc, hipStream_t st) {
  hipLaunchKernelGGL(k_grad_partial, dim3((unsigned)((n + 255) / 256), nseg), dim3(256), 0, st, p, lam, n, nf, ni, k2,
                     nseg, part);
  FWI_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_grad_accum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, part, nseg, n, first, acc);
  FWI_LAUNCH_CHECK();
}

void launch_grad_chain(long n, const c128* acc, double dV, c128 ik0r, const double* c, const double* alpha, c128* g,
                       double* gc, double* ga, hipStream_t st) {
  hipLaunchKernelGGL(k_grad_chain, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, acc, n, dV, ik0r, c, alpha,
                     g, gc, ga);
  FWI_LAUNCH_CHECK();
}

static TvGeo tvgeo(const Geo& g) { return TvGeo{g.dim, g.nx, g.ny, g.nz}; }

void launch_tv_grad(const Geo& g, const c128* m, c128* out, hipStream_t st) {
  const long n = g.n();
  hipLaunchKernelGGL(k_tv_grad, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, tvgeo(g), m, out);
  FWI_LAUNCH_CHECK();
}
void launch_tv_gradT(const Geo& g, const c128* a, double alpha, double beta, c128* out, hipStream_t st) {
  const long n = g.n();
  hipLaunchKernelGGL(k_tv_gradT, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, tvgeo(g), a, alpha, beta, out);
  FWI_LAUNCH_CHECK();
}
int launch_tv_shrink_dual(const Geo& g, const c128* gm, double tau, double dual, c128* gout, c128* u, double* tvp,
                          hipStream_t st) {
  const long n = g.n();
  const unsigned nb = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_tv_shrink_dual, dim3(nb), dim3(256), 0, st, tvgeo(g), gm, tau, dual, gout, u, tvp);
  FWI_LAUNCH_CHECK();
  return (int)nb;
}
void launch_lincomb(long n, double a, const c128* x, double b, const c128* y, double c, const c128* z, c128* out,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_lincomb, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, a, x, b, y, c, z, out);
  FWI_LAUNCH_CHECK();
}
int dot_blocks(long n) {
  long b = (n + 255) / 256;
  return (int)(b > 512 ? 512 : (b < 1 ? 1 : b));
}
void launch_dot_re(long n, const c128* x, const c128* y, double* part, double* out, hipStream_t st) {
  const int nb = dot_blocks(n);
  hipLaunchKernelGGL(k_dot_re_partial, dim3(nb), dim3(256), 0, st, n, x, y, part);
  FWI_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_sum_partial, dim3(1), dim3(64), 0, st, nb, part, out);
  FWI_LAUNCH_CHECK();
}
void launch_sum(int nb, const double* part, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_partial, dim3(1), dim3(64), 0, st, nb, part, out);
  FWI_LAUNCH_CHECK();
}
void launch_cg_step1(long n, const double* sc, c128* x, c128* r, const c128* p, const c128* Ap, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_step1, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, sc, x, r, p, Ap);
  FWI_LAUNCH_CHECK();
}
void launch_cg_step2(long n, const double* sc, const c128* r, c128* p, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_step2, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, sc, r, p);
  FWI_LAUNCH_CHECK();
}
void launch_copy_scalar(const double* in, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(64), 0, st, in, out);
  FWI_LAUNCH_CHECK();
}

// Coarse inversion mesh (factor r): forward cell (ix, iy, iz) takes coarse
// cell (ix / r, iy / r, iz / r); the restriction sums each coarse cell's
// forward cells in a fixed order (the adjoint of the prolongation).
__global__ void k_prolong(TvGeo g, int r, const c128* __restrict__ mc, c128* __restrict__ mf) {
  const long n = (long)g.nx * g.ny * g.nz;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int ix = (int)(i % g.nx), iy = (int)((i / g.nx) % g.ny), iz = (int)(i / ((long)g.nx * g.ny));
  const int cx = (g.nx + r - 1) / r, cy = g.dim == 3 ? (g.ny + r - 1) / r : 1;
  const int jy = g.dim == 3 ? iy / r : 0;
  mf[i] = mc[((long)(iz / r) * cy + jy) * cx + ix / r];
}
__global__ void k_restrict(TvGeo g, int r, const c128* __restrict__ gf, c128* __restrict__ gcv) {
  const int cx = (g.nx + r - 1) / r, cy = g.dim == 3 ? (g.ny + r - 1) / r : 1, cz = (g.nz + r - 1) / r;
  const long nc = (long)cx * cy * cz;
  const long j = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nc) return;
  const int jx = (int)(j % cx), jy = (int)((j / cx) % cy), jz = (int)(j / ((long)cx * cy));
  const int ry = g.dim == 3 ? r : 1;
  c128 s = mk(0.0, 0.0);
  for (int a = 0; a < r; ++a) {
    const int iz = jz * r + a;
    if (iz >= g.nz) break;
    for (int b = 0; b < ry; ++b) {
      const int iy = g.dim == 3 ? jy * r + b : 0;
      if (iy >= g.ny) break;
      for (int e = 0; e < r; ++e) {
        const int ix = jx * r + e;
        if (ix >= g.nx) break;
        s = s + gf[((long)iz * g.ny + iy) * g.nx + ix];
      }
    }
  }
  gcv[j] = s;
}
void launch_prolong(const Geo& g, int r, const c128* mc, c128* mf, hipStream_t st) {
  const long n = g.n();
  hipLaunchKernelGGL(k_prolong, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, tvgeo(g), r, mc, mf);
  FWI_LAUNCH_CHECK();
}
void launch_restrict(const Geo& g, int r, const c128* gf, c128* gcv, hipStream_t st) {
  const long nc = (long)((g.nx + r - 1) / r) * (g.dim == 3 ? (g.ny + r - 1) / r : 1) * ((g.nz + r - 1) / r);
  hipLaunchKernelGGL(k_restrict, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, tvgeo(g), r, gf, gcv);
  FWI_LAUNCH_CHECK();
}

// out[i] = conj(in[i]) (transmit weights into the form the NN product takes)
__global__ void k_conj_c128(long count, const c128* __restrict__ in, c128* __restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = conj(in[i]);
}
void launch_conj_c128(long count, const c128* in, c128* out, hipStream_t st) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_conj_c128, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, count, in, out);
  FWI_LAUNCH_CHECK();
}

// rf[b] = l0 + b / per: frequency index of RHS b of a batch that holds `per`
// RHS per frequency, frequency-major
__global__ void k_fill_rfreq(int B, int per, int l0, int* __restrict__ rf) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) rf[b] = l0 + b / per;
}
void launch_fill_rfreq(int B, int per, int l0, int* rf, hipStream_t st) {
  if (B == 0) return;
  hipLaunchKernelGGL(k_fill_rfreq, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, st, B, per, l0, rf);
  FWI_LAUNCH_CHECK();
}

}  // namespace fwi

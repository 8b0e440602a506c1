// Batched GMRES kernels: classical Gram-Schmidt Arnoldi with FP64 inner
// products (two-stage, fixed-order reductions, no floating-point atomics),
// device-side complex Givens rotations and per-RHS convergence masks. The
// Gram-Schmidt update itself and the solution update run inside the first FFT
// pass of the next matvec (fft_passes.hpp); the kernels here reduce, rotate,
// test and, on the graph-replayed path, update the solution.
#include "krylov.hpp"

namespace fwi {

constexpr int KT = 256;  // threads per block of the vector kernels

// Blocks per RHS of the vector kernels: chunks of at most EPT * KT = 4096
// elements, EPT per thread held in registers.
constexpr int EPT = 16;
int krylov_nblk(long n) {
  long nb = (n + EPT * KT - 1) / (EPT * KT);
  return (int)(nb < 1 ? 1 : nb);
}

// The inner-product kernel (used when the operator's last pass cannot
// produce them) keeps the block's EPT elements per thread of the new vector
// in registers and streams the basis vectors one after another, each with EPT
// independent coalesced loads per thread (indices clamped, values masked, so
// the loads are not behind branches); per-vector sums are reduced wave by
// wave in a fixed order.

// ------------------------------------------------------------------ dots ---
// dotp[b][blk][i] = sum over the block's chunk of conj(V_i) . V_{j+1}, i <= j
template <typename T, int JM>
__global__ void __launch_bounds__(KT) k_dots(const cplx<T>* __restrict__ V, long vs, int j, long n, int chunk,
                                             const int* __restrict__ active, const cplx<T>* __restrict__ vscale,
                                             int B, c128* __restrict__ dotp, int nblk) {
  const int b = blockIdx.y;
  if (!active[b]) return;
  const int t = threadIdx.x;
  const long off = (long)b * n;
  const long e0 = (long)blockIdx.x * chunk;
  const int cnt = (int)min((long)chunk, n - e0);
  const cplx<T>* W = V + (long)(j + 1) * vs + off + e0;
  double wx[EPT], wy[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int e = t + q * KT;
    const cplx<T> w = W[e < cnt ? e : cnt - 1];
    wx[q] = e < cnt ? (double)w.x : 0.0;
    wy[q] = e < cnt ? (double)w.y : 0.0;
  }
  __shared__ double red[2][JM + 1][KT / 64];
  const int lane = t & 63, wvi = t >> 6;
  for (int i = 0; i <= j; ++i) {
    const cplx<T>* Vi = V + (long)i * vs + off + e0;
    cplx<T> vv[EPT];  // all loads of the vector issued before any arithmetic
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = t + q * KT;
      vv[q] = Vi[e < cnt ? e : cnt - 1];
    }
    double r = 0.0, m = 0.0;
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const double vx = vv[q].x, vy = vv[q].y;  // wx, wy are zero past the chunk
      r = fma(vx, wx[q], r);
      r = fma(vy, wy[q], r);
      m = fma(vx, wy[q], m);
      m = fma(-vy, wx[q], m);
    }
    r = wave_sum(r);
    m = wave_sum(m);
    if (lane == 0) {
      red[0][i][wvi] = r;
      red[1][i][wvi] = m;
    }
  }
  __syncthreads();
  if (t <= j) {
    double r = 0.0, m = 0.0;
#pragma unroll
    for (int w = 0; w < KT / 64; ++w) {
      r += red[0][t][w];
      m += red[1][t][w];
    }
    const double sc = (double)vscale[(long)t * B + b].x;  // stored V_i = basis vector / sc
    dotp[((long)b * nblk + blockIdx.x) * (JM + 1) + t] = mk(sc * r, sc * m);
  }
}

// Column j of H: h_i = sum of the ndot inner-product parts of RHS b, wave w
// reducing vectors i = w, w + 4, ..., each lane a fixed subset of parts, then
// a fixed-order wave sum. The classical Gram-Schmidt coefficients
// coef_i = -h_i * scale_i (the update uses the stored, unnormalised vectors)
// go to hcoef for the first pass of the next matvec. Zeroes the active count
// that k_givens accumulates.
template <typename T, int JM>
__global__ void __launch_bounds__(KT) k_hsum(int j, int B, const int* __restrict__ active,
                                             const cplx<T>* __restrict__ vscale, const c128* __restrict__ dotp,
                                             int ndot, c128* __restrict__ H, c128* __restrict__ hcoef,
                                             int* __restrict__ counters) {
  const int b = blockIdx.x;
  if (b == 0 && threadIdx.x == 0) counters[0] = 0;
  if (!active[b]) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int i = w; i <= j; i += KT / 64) {
    double r = 0.0, m = 0.0;
    for (int k = lane; k < ndot; k += 64) {
      const c128 d = dotp[((long)b * ndot + k) * (JM + 1) + i];
      r += d.x;
      m += d.y;
    }
    r = wave_sum(r);
    m = wave_sum(m);
    if (lane == 0) {
      H[((long)b * (JM + 1) + i) * JM + j] = mk(r, m);
      const double sc = (double)vscale[(long)i * B + b].x;
      hcoef[(long)b * (JM + 1) + i] = mk(-(r * sc), -(m * sc));
    }
  }
}

// One workgroup per RHS: finish column j (norm of the orthogonalised vector
// from its per-row sums, summed by the whole workgroup in a fixed order;
// previous rotations, new rotation), update the residual estimate and the
// convergence mask, count the RHS still active.
template <typename T, int JM>
__global__ void __launch_bounds__(KT) k_givens(int j, int B, int rows, const double* __restrict__ rowpart,
                                               int* __restrict__ active, c128* __restrict__ H,
                                               double* __restrict__ cs, c128* __restrict__ sn,
                                               c128* __restrict__ gv, const double* __restrict__ target,
                                               int* __restrict__ ncol, int* __restrict__ iters,
                                               cplx<T>* __restrict__ vscale_next, int* __restrict__ counters) {
  __shared__ double red[KT / 64];
  const int b = blockIdx.x;
  if (b >= B || !active[b]) return;  // uniform per workgroup
  double s2 = 0.0;
  for (int k = threadIdx.x; k < rows; k += KT) s2 += rowpart[(long)b * rows + k];
  s2 = block_sum<KT>(s2, red);
  if (threadIdx.x != 0) return;
  const double hn = sqrt(s2);
  c128* col = H + (long)b * (JM + 1) * JM + j;  // col[i*JM] = H[i][j]
  for (int i = 0; i < j; ++i) {
    const c128 a = col[i * JM], c2 = col[(i + 1) * JM];
    const double c = cs[b * JM + i];
    const c128 s = sn[b * JM + i];
    col[i * JM] = c * a + s * c2;
    col[(i + 1) * JM] = c * c2 - conj(s) * a;
  }
  const c128 a = col[j * JM];
  const double aa = sqrt(norm2(a));
  const double nu = sqrt(aa * aa + hn * hn);
  if (nu == 0.0) {
    // A v_j = 0 after orthogonalisation: column j is zero and adds nothing to
    // the least-squares problem, so it is left out (ncol stays j) and the RHS
    // stops with the solution of the first j columns
    iters[b] += 1;
    active[b] = 0;
    return;
  }
  double c;
  c128 s;
  if (aa == 0.0) {
    c = 0.0;
    s = mk(1.0, 0.0);
  } else {
    c = aa / nu;
    s = (hn / (nu * aa)) * a;
  }
  cs[b * JM + j] = c;
  sn[b * JM + j] = s;
  col[j * JM] = c * a + hn * s;
  col[(j + 1) * JM] = mk(0.0, 0.0);
  const c128 g = gv[b * (JM + 1) + j];
  gv[b * (JM + 1) + j] = c * g;
  const c128 g1 = (-1.0) * (conj(s) * g);
  gv[b * (JM + 1) + j + 1] = g1;
  ncol[b] = j + 1;
  iters[b] += 1;
  const double res = sqrt(norm2(g1));
  if (res <= target[b] || !(hn > 1e-300) || nu == 0.0) {
    active[b] = 0;
  } else {
    vscale_next[b] = mk((T)(1.0 / hn), (T)0);
    atomicAdd(counters, 1);
  }
}

// nrmp[b][blk] = sum of the block's share of the per-row partials of RHS b.
__global__ void __launch_bounds__(KT) k_rows_norm(const double* __restrict__ rowpart, int rows, int per,
                                                  double* __restrict__ nrmp, int nblk) {
  __shared__ double red[KT / 64];
  const int b = blockIdx.y;
  const int r0 = blockIdx.x * per;
  const int r1 = min(rows, r0 + per);
  const double* rp = rowpart + (long)b * rows;
  double acc = 0.0;
  for (int r = r0 + threadIdx.x; r < r1; r += KT) acc += rp[r];
  const double s = block_sum<KT>(acc, red);
  if (threadIdx.x == 0) nrmp[(long)b * nblk + blockIdx.x] = s;
}

// Start of a cycle: residual norms, activity, stopping targets.
template <typename T, int JM>
__global__ void __launch_bounds__(1024) k_cycle_init(int B, int nblk, int first, double rtol, double inner_rtol,
                                                     const double* __restrict__ nrmp, double* __restrict__ rnorm,
                                                     double* __restrict__ bnorm, double* __restrict__ target,
                                                     double* __restrict__ rscale, int* __restrict__ active,
                                                     int* __restrict__ ncol, c128* __restrict__ gv,
                                                     int* __restrict__ counters, double* __restrict__ maxrel,
                                                     cplx<T>* __restrict__ vscale0) {
  __shared__ double red[1024 / 64];
  __shared__ double redm[1024 / 64];
  double cnt = 0.0, mx = 0.0;
  for (int b = threadIdx.x; b < B; b += blockDim.x) {
    double s2 = 0.0;
    for (int k = 0; k < nblk; ++k) s2 += nrmp[(long)b * nblk + k];
    const double rn = sqrt(s2);
    if (first) bnorm[b] = rn;
    const double bn = bnorm[b];
    rnorm[b] = rn;
    ncol[b] = 0;
    gv[(long)b * (JM + 1)] = mk(1.0, 0.0);
    const int act = rn > rtol * bn;
    active[b] = act;
    const double rel = bn > 0.0 ? rn / bn : 0.0;
    mx = fmax(mx, rel);
    if (act) {
      cnt += 1.0;
      // relative reduction this cycle must reach for |r| <= rtol |b|; an inner
      // (complex64) cycle aims at half of it, since its residual estimate
      // is not the FP64 residual that the next cycle start checks, and stops
      // no later than at inner_rtol
      double tg = rtol * bn / rn;
      if (inner_rtol > 0.0) tg *= 0.5;
      if (inner_rtol > tg) tg = inner_rtol;
      target[b] = tg;
      rscale[b] = 1.0 / rn;
      vscale0[b] = mk((T)(1.0 / rn), (T)0);  // V_0 holds r unscaled
    }
  }
  const double tot = block_sum<1024>(cnt, red);
  // max-reduce
  double m = mx;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) redm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mm = 0.0;
    for (int w = 0; w < (int)(blockDim.x / 64); ++w) mm = fmax(mm, redm[w]);
    maxrel[0] = mm;
    counters[0] = (int)tot;
    counters[1] = (int)tot;
  }
}

// Back-substitution R y = g for each RHS (k = ncol columns).
template <typename T, int JM>
__global__ void k_backsolve(int B, const int* __restrict__ ncol, const c128* __restrict__ H,
                            const c128* __restrict__ gv, c128* __restrict__ y, const double* __restrict__ rnorm,
                            const cplx<T>* __restrict__ vscale) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const int k = ncol[b];
  const c128* Hb = H + (long)b * (JM + 1) * JM;
  for (int i = k - 1; i >= 0; --i) {
    c128 acc = gv[(long)b * (JM + 1) + i];
    for (int l = i + 1; l < k; ++l) acc = acc - Hb[i * JM + l] * y[(long)b * JM + l];
    const c128 d = Hb[i * JM + i];
    const double dn = norm2(d);
    // acc / d (a zero diagonal cannot occur for a kept column; guarded anyway)
    y[(long)b * JM + i] = dn > 0.0 ? mk((acc.x * d.x + acc.y * d.y) / dn, (acc.y * d.x - acc.x * d.y) / dn)
                                   : mk(0.0, 0.0);
  }
  // the basis is normalised by |r| (cycle start) and stored with scales
  for (int i = 0; i < k; ++i) {
    const double sc = rnorm[b] * (double)vscale[(long)i * B + b].x;
    const c128 v = y[(long)b * JM + i];
    y[(long)b * JM + i] = mk(sc * v.x, sc * v.y);
  }
}

// x_b += sum_{i < ncol_b} y_i V_i (FP64 accumulation, y from k_backsolve);
// first: x_b is not read (the first cycle starts from x = 0), and RHS that
// did no step get 0.
template <typename T, int JM>
__global__ void __launch_bounds__(KT) k_xupdate(const cplx<T>* __restrict__ V, long vs, long n,
                                                const int* __restrict__ ncol, const c128* __restrict__ y,
                                                c128* __restrict__ x, int first) {
  const int b = blockIdx.y;
  const int k = ncol[b];
  if (k == 0) {
    if (first)
      for (long e = (long)blockIdx.x * KT + threadIdx.x; e < n; e += (long)gridDim.x * KT) x[(long)b * n + e] = mk(0.0, 0.0);
    return;
  }
  __shared__ c128 yc[JM];
  if (threadIdx.x < k) yc[threadIdx.x] = y[(long)b * JM + threadIdx.x];
  __syncthreads();
  const long off = (long)b * n;
  for (long e = (long)blockIdx.x * KT + threadIdx.x; e < n; e += (long)gridDim.x * KT) {
    c128 acc = first ? mk(0.0, 0.0) : x[off + e];
#pragma unroll
    for (int i = 0; i < JM; ++i) {
      if (i < k) {
        const cplx<T> v = V[(long)i * vs + off + e];
        acc = cfma(yc[i], mk((double)v.x, (double)v.y), acc);
      }
    }
    x[off + e] = acc;
  }
}

// Largest and total iteration count of a solve, folded into st[0] (max) and
// st[1] (sum) so the host reads them once per call.
__global__ void __launch_bounds__(KT) k_iter_stats(int B, const int* __restrict__ iters,
                                                   unsigned long long* __restrict__ st) {
  __shared__ unsigned long long smax[KT], ssum[KT];
  unsigned long long mx = 0, s = 0;
  for (int b = threadIdx.x; b < B; b += KT) {
    const unsigned long long v = (unsigned long long)iters[b];
    mx = v > mx ? v : mx;
    s += v;
  }
  smax[threadIdx.x] = mx;
  ssum[threadIdx.x] = s;
  __syncthreads();
  for (int o = KT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      smax[threadIdx.x] = smax[threadIdx.x] > smax[threadIdx.x + o] ? smax[threadIdx.x] : smax[threadIdx.x + o];
      ssum[threadIdx.x] += ssum[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicMax(&st[0], smax[0]);
    atomicAdd(&st[1], ssum[0]);
  }
}

__global__ void k_zero_u64(unsigned long long* p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0;
}

void launch_iter_stats(int B, const int* iters, unsigned long long* st, hipStream_t s) {
  hipLaunchKernelGGL(k_iter_stats, dim3(1), dim3(KT), 0, s, B, iters, st);
  FWI_LAUNCH_CHECK();
}

void launch_zero_u64(int count, unsigned long long* p, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3((count + 255) / 256), dim3(256), 0, s, p, count);
  FWI_LAUNCH_CHECK();
}

__global__ void k_zero_int(int* p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0;
}

__global__ void k_fill_zero_c128(long count, c128* p) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = mk(0.0, 0.0);
}
__global__ void k_copy_c128(long count, const c128* __restrict__ in, c128* __restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = in[i];
}

void launch_fill_zero_c128(long count, c128* p, hipStream_t st) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_fill_zero_c128, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, count, p);
  FWI_LAUNCH_CHECK();
}
void launch_copy_c128(long count, const c128* in, c128* out, hipStream_t st) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_copy_c128, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, count, in, out);
  FWI_LAUNCH_CHECK();
}

// ------------------------------------------------------------- launchers ---
static unsigned vec_blocks(long n) {
  long b = (n + KT * 4 - 1) / (KT * 4);
  if (b > 1024) b = 1024;
  return (unsigned)(b < 1 ? 1 : b);
}

#define FWI_JM_SWITCH(JM_RT, ...)                                            \
  switch (JM_RT) {                                                           \
    case 8: { constexpr int JMC = 8; __VA_ARGS__; } break;                   \
    case 16: { constexpr int JMC = 16; __VA_ARGS__; } break;                 \
    case 32: { constexpr int JMC = 32; __VA_ARGS__; } break;                 \
    default: throw Error(-6, "unsupported GMRES basis capacity");            \
  }

template <typename T>
void krylov_rows_norm(const KrylovState<T>& s, const double* rowpart, int rows, hipStream_t st) {
  const int per = (rows + s.nblk - 1) / s.nblk;
  hipLaunchKernelGGL(k_rows_norm, dim3(s.nblk, s.B), dim3(KT), 0, st, rowpart, rows, per, s.nrmp, s.nblk);
  FWI_LAUNCH_CHECK();
}

template <typename T>
void krylov_cycle_init(const KrylovState<T>& s, int first, double rtol, double inner_rtol, hipStream_t st) {
  FWI_JM_SWITCH(s.JM, hipLaunchKernelGGL((k_cycle_init<T, JMC>), dim3(1), dim3(1024), 0, st, s.B, s.nblk, first, rtol,
                                          inner_rtol, s.nrmp, s.rnorm, s.bnorm, s.target, s.rscale, s.active, s.ncol,
                                          s.gv, s.counters, s.maxrel, s.vscale));
  FWI_LAUNCH_CHECK();
}

template <typename T>
void krylov_dots(const KrylovState<T>& s, int j, hipStream_t st) {
  const int po = sizeof(T) == 8 ? KC_COUNT : 0;
  prof_begin(KC_DOTS + po, st);
  FWI_JM_SWITCH(s.JM, FWI_TIMED_LAUNCH((k_dots<T, JMC>), dim3(s.nblk, s.B), dim3(KT), 0, st, s.V, s.vstride(), j,
                                          s.n, s.chunk, s.active, s.vscale, s.B, s.dotp, s.nblk));
  FWI_LAUNCH_CHECK();
  prof_end(KC_DOTS + po, st, (j + 2) * (double)s.n * sizeof(cplx<T>), 0.0, true, s.B);
}

template <typename T>
void krylov_hsum(const KrylovState<T>& s, int j, int ndot, hipStream_t st) {
  FWI_JM_SWITCH(s.JM, hipLaunchKernelGGL((k_hsum<T, JMC>), dim3(s.B), dim3(KT), 0, st, j, s.B, s.active, s.vscale,
                                          s.dotp, ndot, s.H, s.hcoef, s.counters));
  FWI_LAUNCH_CHECK();
}

template <typename T>
void krylov_givens(const KrylovState<T>& s, int j, const double* rowpart, int rows, hipStream_t st) {
  FWI_JM_SWITCH(s.JM, hipLaunchKernelGGL((k_givens<T, JMC>), dim3(s.B), dim3(KT), 0, st,
                                          j, s.B, rows, rowpart, s.active, s.H, s.cs, s.sn, s.gv, s.target, s.ncol,
                                          s.iters, s.vscale + (long)(j + 1) * s.B, s.counters));
  FWI_LAUNCH_CHECK();
}

template <typename T>
void krylov_backsolve(const KrylovState<T>& s, hipStream_t st) {
  FWI_JM_SWITCH(s.JM, hipLaunchKernelGGL((k_backsolve<T, JMC>), dim3((s.B + 63) / 64), dim3(64), 0, st, s.B,
                                          s.ncol, s.H, s.gv, s.y, s.rnorm, s.vscale));
  FWI_LAUNCH_CHECK();
}

template <typename T>
void krylov_xupdate(const KrylovState<T>& s, c128* x, int first, hipStream_t st) {
  FWI_JM_SWITCH(s.JM, hipLaunchKernelGGL((k_xupdate<T, JMC>), dim3(vec_blocks(s.n), s.B), dim3(KT), 0, st, s.V,
                                          s.vstride(), s.n, s.ncol, s.y, x, first));
  FWI_LAUNCH_CHECK();
}

template <typename T>
void krylov_finish_cycle(const KrylovState<T>& s, c128* x, int first, hipStream_t st) {
  krylov_backsolve(s, st);
  krylov_xupdate(s, x, first, st);
}

template <typename T>
void krylov_reset_iters(const KrylovState<T>& s, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_int, dim3((s.B + 255) / 256), dim3(256), 0, st, s.iters, s.B);
  FWI_LAUNCH_CHECK();
}

#define FWI_INST(T)                                                                            \
  template void krylov_rows_norm<T>(const KrylovState<T>&, const double*, int, hipStream_t);   \
  template void krylov_cycle_init<T>(const KrylovState<T>&, int, double, double, hipStream_t); \
  template void krylov_dots<T>(const KrylovState<T>&, int, hipStream_t);                        \
  template void krylov_hsum<T>(const KrylovState<T>&, int, int, hipStream_t);                   \
  template void krylov_givens<T>(const KrylovState<T>&, int, const double*, int, hipStream_t);  \
  template void krylov_backsolve<T>(const KrylovState<T>&, hipStream_t);                       \
  template void krylov_xupdate<T>(const KrylovState<T>&, c128*, int, hipStream_t);             \
  template void krylov_finish_cycle<T>(const KrylovState<T>&, c128*, int, hipStream_t);        \
  template void krylov_reset_iters<T>(const KrylovState<T>&, hipStream_t);
FWI_INST(float)
FWI_INST(double)

}  // namespace fwi

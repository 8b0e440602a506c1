/*
 * fwi.h - C ABI of the MI355X (gfx950) hot path of TV-regularized
 * frequency-domain full-waveform inversion for single-sided linear arrays.
 *
 * The method (Guo, Auerbach, Eldar): the total field of transmit i at
 * frequency l solves the volume integral equation (Eq. 5)
 *     p = p0 + k0^2 int_V G(x, x') m(x') p(x') dx',
 * the scattered data are P^s_{i,j,l} = k0^2 int G m p at receiver j (Eq. 4),
 * the Green's-function product is an FFT convolution and the system is
 * solved by a Krylov method (Sec. IV-A), the gradient and Jacobian products
 * come from forward and adjoint fields (Eq. 15-17), and the model is updated
 * by ADMM with an isotropic TV prior (Eq. 7-14, Algorithm 1).
 *
 * Discretisation (the paper says only "after discretization"): square/cubic
 * cells of size dx, pulse basis, collocation at cell centres, cell integral of
 * G over the equal-area disk / equal-volume ball (Richmond), point elements on
 * the top face z = 0, point receivers with the midpoint rule. Time convention
 * e^{-i omega t}: complex values are the conjugates of the paper's.
 *
 * Conventions for every entry point
 *  - Grids are depth-major: index ((iz * ny) + iy) * nx + ix, x fastest; ny = 1
 *    in 2D. Cell centres at ((ix+1/2)dx, (iy+1/2)dx, (iz+1/2)dx).
 *  - Complex arrays are interleaved (re, im): complex128 = 2 doubles,
 *    complex64 = 2 floats.
 *  - Data arrays are [nf][ne][ne] with layout [l][i][j] (transmit i, receiver j).
 *  - Fields / RHS arrays are [nf][ne][n] (frequency-major, then transmit).
 *  - fwi_problem and its freq_hz / elem_xyz arrays, option/param structs and
 *    scalar outputs (misfit, stats, report) are HOST memory. Every grid, data,
 *    field and state array argument is DEVICE memory on the context's device.
 *  - Calls are enqueued on the context's HIP stream; they return after the
 *    host-visible scalars (misfit, stats, report) are known, which requires
 *    synchronising that stream. Array outputs are complete when the call
 *    returns FWI_OK.
 *  - The library never frees or retains caller memory; it reads inputs as
 *    const and writes only the named outputs and its workspace.
 *  - Return codes are 0 (FWI_OK) or a negative FWI_E_* code; no exception
 *    crosses the ABI. fwi_last_error() gives a message for the last failure
 *    on that context. One context per stream; contexts are not thread-safe.
 */
#ifndef FWI_H
#define FWI_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FWI_OK 0
#define FWI_E_INVAL (-1)       /* invalid argument (shape, pointer, value) */
#define FWI_E_NOMEM (-2)       /* caller workspace too small / allocation failed */
#define FWI_E_NOCONV (-3)      /* a solve hit max_iter; outputs are still written */
#define FWI_E_NONFINITE (-4)   /* NaN/Inf in an input or a residual */
#define FWI_E_DEVICE (-5)      /* HIP runtime error */
#define FWI_E_UNSUPPORTED (-6) /* size or mode outside what the library implements */

#define FWI_FP64 0          /* complex128 everywhere */
#define FWI_FP32_REFINE 1   /* complex64 Krylov solves inside FP64-residual refinement */

typedef struct fwi_ctx fwi_ctx;

/* Problem statement (Sec. II): grid of cells, constant-density background
 * of speed of sound c0 (and attenuation alpha0, below), frequencies and
 * element positions on the top face z = 0.
 * Each axis must satisfy 1 <= n <= 512 (padded FFT length 2^a 3^b <= 1024). */
typedef struct fwi_problem {
  int dim;                 /* 2 or 3 */
  int nx, ny, nz;          /* cells: lateral x, elevation y (1 in 2D), depth z */
  double dx;               /* cell size [m] */
  double c0;               /* background speed of sound [m/s] */
  int nf;                  /* number of frequencies */
  const double* freq_hz;   /* host [nf], > 0 */
  int ne;                  /* number of elements (transmit set = receive set) */
  const double* elem_xyz;  /* host [ne][3] positions [m]; z must be 0 */
  /* Element aperture (Sec. V: finite elements; Eq. 4 integrates over the
   * receiver region): a rectangle on the top face centred at elem_xyz, width
   * along x, height along y (3D only). Each element transmits and receives as
   * the average of the point-source field over its aperture, by an
   * elem_quad-point Gauss-Legendre rule per direction (1..16). Zero width and
   * height: point elements (elem_quad ignored). */
  double elem_width;       /* [m], >= 0 */
  double elem_height;      /* [m], >= 0, 0 in 2D */
  int elem_quad;
  /* Background attenuation alpha0 [Np/m/Hz] >= 0 (Sec. II: kappa_0 from c0 and
   * alpha0; the background wavenumber is then complex and decaying, and the
   * 2D Green's function takes Hankel functions of complex argument). 0: the
   * lossless background. */
  double alpha0;
} fwi_problem;

/* Solver options (Sec. IV-A: Krylov solve of the discretised Eq. 5). */
typedef struct fwi_solve_opts {
  int precision;        /* FWI_FP64 or FWI_FP32_REFINE */
  double rtol;          /* target ||b - A x|| / ||b|| in FP64, per RHS */
  int max_iter;         /* cap on Krylov iterations per RHS (all cycles) */
  int restart;          /* GMRES basis length: 8, 16 or 32 */
  int max_refine;       /* FP32_REFINE: cap on refinement steps */
  double inner_rtol;    /* FP32_REFINE: floor of each inner cycle's relative target; a cycle
                           stops at the larger of this and half the reduction that
                           rtol still needs (the FP64 residual of the next cycle start
                           decides convergence) */
  int max_rhs;          /* cap on RHS per batched solve (0: all frequencies at once) */
  int check_every;      /* iterations between host convergence checks (>= 1); a check
                           is read after the next step is enqueued, so at most one
                           fully masked step follows convergence */
  int reciprocity_adjoint; /* 1: adjoint fields as sum_j conj(r_ij) p_j (no adjoint solves) */
  int fields_c64;       /* fields_out of the forward entries as complex64 (1) or complex128 (0);
                           the solves themselves are unchanged */
  int tx_chunk;         /* > 0 and < the transmits per frequency: solve the transmits of one
                           frequency at a time in chunks of tx_chunk (the workspace then holds
                           tx_chunk RHS instead of a frequency group); 0: whole frequencies */
} fwi_solve_opts;

/* Per-call statistics (host struct, written when non-NULL). */
typedef struct fwi_stats {
  int iterations;          /* max Krylov iterations over the RHS of the call */
  int cycles;              /* max restart cycles / refinement steps of a batch */
  int unconverged;         /* RHS that did not reach rtol */
  double max_rel_residual; /* max final FP64 relative residual */
  long long solves;        /* right-hand sides solved (forward + adjoint) */
  long long matvecs;       /* operator applications summed over RHS */
  double t_setup_ms;       /* contrast, Green spectra, incident fields */
  double t_solve_ms;       /* Krylov solves */
  double t_total_ms;       /* whole call */
} fwi_stats;

/* ADMM parameters (Eq. 8-14, Algorithm 1). */
typedef struct fwi_admm_params {
  double lambda;      /* TV weight */
  double rho;         /* augmented-Lagrangian penalty */
  double gamma;       /* reference-model weight (ignored when m_ref is NULL) */
  int n_cg;           /* CG iterations on the normal equations (Eq. 11-12) */
  double data_scale;  /* s multiplying the data term; <= 0 selects 1/||d_obs||^2 */
  double dual_step;   /* u += dual_step (g - grad m); the paper prints rho */
  int inv_factor;     /* inversion mesh (Sec. IV: coarser than the forward mesh): <= 1 the forward
                         mesh; r > 1 cells of r x r (x r) forward cells (ceil per axis, ragged last
                         cells), piecewise-constant model, Jacobian J P. m, g, u, m_ref then live on
                         the inversion mesh ([ceil(nz/r)][ceil(ny/r)][ceil(nx/r)]) */
} fwi_admm_params;

typedef struct fwi_admm_report {
  double misfit;   /* 1/2 ||F(m_k) - d_obs||^2 at the input model */
  double tv;       /* ||grad m_{k+1}||_{1,2} */
  double dm_norm;  /* ||m_{k+1} - m_k|| */
} fwi_admm_report;

/* ---------------------------------------------------------------- context */
/* Create a context on HIP device `device` enqueuing on `hip_stream` (a
 * hipStream_t; NULL = default stream). The context owns only caches (twiddle
 * tables, Green spectra and incident fields of the last problem) and, when no
 * caller workspace is set, an internal workspace. */
int fwi_create(fwi_ctx** out, int device, void* hip_stream);
void fwi_destroy(fwi_ctx* ctx);
const char* fwi_last_error(const fwi_ctx* ctx);
int fwi_set_stream(fwi_ctx* ctx, void* hip_stream);
/* Strided FFT passes address each plane through 32-bit buffer views and fall
 * back to 64-bit addressing for planes of 2 GiB or more. wide = 1 forces the
 * 64-bit path for every later call (a testing aid for that path; results are
 * the same), 0 restores the automatic choice. FWI_E_INVAL for other values. */
int fwi_set_addressing(fwi_ctx* ctx, int wide);
/* 3D complex64 operator (Sec. IV-A, the convolution of Eq. 5 by FFT): with
 * on = 1, on grids whose padded lateral and elevation lengths allow it
 * (Lx/4, Ly/2 in {(64, 128), (32, 64)}), one kernel per z-plane does the
 * lateral and elevation transforms together, in four lateral by two elevation
 * frequency classes, so the intermediate between them never goes to memory;
 * the padded spectrum and the cached complex64 kernel spectrum are then
 * stored class-major (same values, permuted). on = 0 (the default) keeps the
 * separate lateral and elevation passes, which are faster on MI355X (the
 * fused kernel holds a plane per workgroup and runs one workgroup per compute
 * unit). Results agree to complex64 rounding. The problem cache is keyed on
 * the setting, so a change rebuilds the spectra at the next call.
 * FWI_E_INVAL for other values. */
int fwi_set_plane_fusion(fwi_ctx* ctx, int on);
void fwi_default_opts(fwi_solve_opts* opts);

/* Host-only argument check; returns FWI_OK or FWI_E_INVAL / FWI_E_UNSUPPORTED.
 * Elements must lie on z = 0 within the lateral extent; frequencies > 0. */
int fwi_validate_problem(const fwi_problem* prob);
/* Padded FFT length used for an axis of n cells (smallest 2^a 3^b >= 2n), 0 if n > 512. */
int fwi_padded_length(int n);

/* Workspace bytes an entry point needs (host-only). entry: 0 forward,
 * 1 adjoint gradient / vjp, 2 ADMM step. Returns FWI_OK and writes *bytes. */
#define FWI_ENTRY_FORWARD 0
#define FWI_ENTRY_GRADIENT 1
#define FWI_ENTRY_ADMM 2
int fwi_workspace_size(const fwi_problem* prob, const fwi_solve_opts* opts, int entry, size_t* bytes);
/* Use caller device memory as workspace (NULL/0 returns to internal allocation).
 * Calls needing more than `bytes` fail with FWI_E_NOMEM. */
int fwi_set_workspace(fwi_ctx* ctx, void* dev_ptr, size_t bytes);

/* ------------------------------------------------------------- hot path */
/* F(m): forward solves for every transmit and frequency and the scattered
 * data (Eq. 3-6). c [n] speed of sound [m/s] > 0, alpha [n] attenuation
 * [Np/m/Hz] >= 0 or NULL (zero), both double. data_out [nf][ne][ne]
 * complex128. fields_out NULL or [nf][ne][n] total fields, complex128, or
 * complex64 when opts->fields_c64 is set. */
int fwi_forward(fwi_ctx* ctx, const fwi_problem* prob, const double* c, const double* alpha,
                const fwi_solve_opts* opts, void* data_out, void* fields_out, fwi_stats* stats);

/* Same as fwi_forward for a contrast m [n] complex128 (Eq. 3). */
int fwi_forward_m(fwi_ctx* ctx, const fwi_problem* prob, const void* m, const fwi_solve_opts* opts,
                  void* data_out, void* fields_out, fwi_stats* stats);

/* Misfit phi = 1/2 ||F(m) - d_obs||^2 and its gradient by adjoint solves
 * with the same operator (Eq. 15-17): g_n = dV sum_l conj(k_l^2) sum_i
 * conj(p_li(x_n) lam_li(x_n)), lam_li = A_l^{-1} sum_j conj(r_lij) p0_lj.
 * d_obs [nf][ne][ne] complex128. misfit_out: host double or NULL.
 * grad_m_out [n] complex128 (d phi/d Re m + i d phi/d Im m) or NULL;
 * grad_c_out, grad_alpha_out [n] double (chain rule) or NULL. */
int fwi_adjoint_gradient(fwi_ctx* ctx, const fwi_problem* prob, const double* c, const double* alpha,
                         const void* d_obs, const fwi_solve_opts* opts, double* misfit_out, void* grad_m_out,
                         double* grad_c_out, double* grad_alpha_out, fwi_stats* stats);

/* Vector-Jacobian product J^H b at contrast m (Eq. 17) via forward and
 * adjoint solves: the backward of fwi_forward_m for automatic differentiation.
 * m [n] complex128, grad_data [nf][ne][ne] complex128, grad_m_out [n] complex128. */
int fwi_vjp(fwi_ctx* ctx, const fwi_problem* prob, const void* m, const void* grad_data,
            const fwi_solve_opts* opts, void* grad_m_out, fwi_stats* stats);

/* fwi_vjp with the forward fields given instead of solved: fields [nf][ne][n]
 * complex128 from an earlier fwi_forward_m at the same m (Eq. 17 needs the
 * forward fields p_li; the adjoint fields are still solved). With the same
 * options the solver is deterministic and a field does not depend on the
 * batch it was solved in, so the result equals fwi_vjp's bit for bit: the
 * stored-fields backward of automatic differentiation, for callers whose
 * fields fit device memory. */
int fwi_vjp_fields(fwi_ctx* ctx, const fwi_problem* prob, const void* m, const void* fields,
                   const void* grad_data, const fwi_solve_opts* opts, void* grad_m_out, fwi_stats* stats);

/* One iteration of Algorithm 1: forward solves at m_k, Gauss-Newton model
 * update by params->n_cg CG iterations on (s J^H J + rho grad^T grad + gamma I)
 * dm = s J^H(d_obs - F(m_k)) + rho grad^T(g + u - grad m_k) + gamma(m_ref - m_k)
 * (Eq. 11-12, the gamma terms dropped when m_ref is NULL), then
 * g = shrink_{lambda/rho}(grad m_{k+1} - u) (Eq. 13-14) and
 * u += dual_step (g - grad m_{k+1}). grad: forward differences, unit spacing,
 * zero at the last index; components ordered x, (y,) z.
 * m_inout [n], g_inout [dim][n], u_inout [dim][n], m_ref [n] or NULL,
 * d_obs [nf][ne][ne]: all complex128, updated in place. */
int fwi_tv_admm_step(fwi_ctx* ctx, const fwi_problem* prob, const fwi_admm_params* params, void* m_inout,
                     void* g_inout, void* u_inout, const void* m_ref, const void* d_obs,
                     const fwi_solve_opts* opts, fwi_admm_report* report, fwi_stats* stats);

/* Algorithm 1 (Sec. III): g_0 = grad m_0, u_0 = 0, then ADMM iterations as in
 * fwi_tv_admm_step (fwi_tv_admm_step_tx when nt > 0: receiver fields
 * recomputed at the first iteration and every born_every-th after it, reused
 * in between; born_every <= 0: first iteration only) until the misfit at the
 * iterate is <= tol * 1/2 ||d_obs||^2 (that iteration's update is kept) or
 * max_iter iterations have run. m_inout [n]: m_0 in, final model out;
 * g_out, u_out [dim][n] (final ADMM variables); rx_fields [nf][ne][n] when
 * nt > 0; all complex128 device arrays. misfit_hist: host double[max_iter]
 * or NULL (misfit at each iterate); iters_done: host int or NULL. stats sum
 * the solves of all iterations. */
int fwi_invert(fwi_ctx* ctx, const fwi_problem* prob, const fwi_admm_params* params, int max_iter, double tol,
               int nt, const void* tx_weights, void* rx_fields, int born_every, void* m_inout, void* g_out,
               void* u_out, const void* m_ref, const void* d_obs, const fwi_solve_opts* opts, double* misfit_hist,
               int* iters_done, fwi_stats* stats);

/* Speed of sound c [n] and attenuation alpha [n] (double, device; either may
 * be NULL) of a contrast m [n] complex128: the inverse of Eq. 1-3 (the
 * positive root of its quadratic in c^2; NaN where none exists). */
int fwi_sos_from_contrast(fwi_ctx* ctx, const fwi_problem* prob, const void* m, double* c_out, double* alpha_out);

/* ------------------------------------------------ synthesised transmits */
/* Transmits other than single elements (Sec. V fires steered plane waves from
 * the array; every element still receives). Transmit t at frequency l drives
 * element e with the complex weight w[l][t][e], so its incident field is
 * sum_e w[l][t][e] p0_le and its total field solves A_l p = that field
 * (Eq. 5). tx_weights: device [nf][nt][ne] complex128, 1 <= nt <= ne (else
 * FWI_E_INVAL; non-finite weights give FWI_E_NONFINITE). data_out
 * [nf][nt][ne] complex128 (Eq. 4, receivers = elements); fields_out NULL or
 * [nf][nt][n] complex128. Workspace as for fwi_adjoint_gradient. */
int fwi_forward_tx(fwi_ctx* ctx, const fwi_problem* prob, const double* c, const double* alpha, int nt,
                   const void* tx_weights, const fwi_solve_opts* opts, void* data_out, void* fields_out,
                   fwi_stats* stats);

/* Misfit and gradient for synthesised transmits by adjoint solves: adjoint
 * sources sum_j conj(r_ltj) p0_lj with r = F - d_obs [nf][nt][ne], adjoint
 * fields by the same operator, g as in fwi_adjoint_gradient with the
 * transmit fields. opts->reciprocity_adjoint must be 0 (the transmit fields
 * are not the receiver fields): else FWI_E_UNSUPPORTED. */
int fwi_adjoint_gradient_tx(fwi_ctx* ctx, const fwi_problem* prob, const double* c, const double* alpha, int nt,
                            const void* tx_weights, const void* d_obs, const fwi_solve_opts* opts,
                            double* misfit_out, void* grad_m_out, double* grad_c_out, double* grad_alpha_out,
                            fwi_stats* stats);

/* fwi_tv_admm_step for synthesised transmits: the Jacobian of Sec. IV-B from
 * the transmit fields at m_k and the receiver fields rx_fields [nf][ne][n]
 * complex128 (device). refresh_rx != 0: rx_fields are recomputed at m_k (ne
 * element solves per frequency, written back); 0: used as given, e.g. kept
 * from an earlier iterate (the paper's Born reuse of the receiver fields).
 * tx_weights as in fwi_forward_tx, d_obs [nf][nt][ne]. */
int fwi_tv_admm_step_tx(fwi_ctx* ctx, const fwi_problem* prob, const fwi_admm_params* params, int nt,
                        const void* tx_weights, void* rx_fields, int refresh_rx, void* m_inout, void* g_inout,
                        void* u_inout, const void* m_ref, const void* d_obs, const fwi_solve_opts* opts,
                        fwi_admm_report* report, fwi_stats* stats);

/* ---------------------------------------------------------- uneven batches */
/* Many independent problems (grids, element counts and frequency counts may
 * all differ) solved together. One refinement cycle of every instance of a
 * wave is captured into one hipGraph (a branch per instance, convergence masks
 * instead of host checks inside the cycle) and the graph is replayed until
 * every right-hand side has converged; instances are grouped into waves that
 * fit 60% of free device memory. Tile variants follow the context's tuning
 * table (fwi_autotune per grid size). Arrays are per instance, as in
 * fwi_adjoint_gradient / fwi_forward; misfit_out is host [ninst]. The caller
 * workspace, if set, must hold the largest wave (else FWI_E_NOMEM). */
typedef struct fwi_batch_stats {
  int waves;               /* instance groups solved one after another */
  int graph_launches;      /* replays of captured cycle graphs */
  int iterations;          /* max Krylov iterations over all RHS */
  int unconverged;         /* RHS that did not reach rtol */
  double max_rel_residual; /* max FP64 relative residual at exit */
  long long solves;        /* right-hand sides solved (forward + adjoint) */
  double t_setup_ms, t_solve_ms, t_total_ms;
} fwi_batch_stats;
int fwi_adjoint_gradient_batch(fwi_ctx* ctx, int ninst, const fwi_problem* probs, const double* const* c,
                               const double* const* alpha, const void* const* d_obs, const fwi_solve_opts* opts,
                               double* misfit_out, void* const* grad_m_out, fwi_batch_stats* stats);
int fwi_forward_batch(fwi_ctx* ctx, int ninst, const fwi_problem* probs, const double* const* c,
                      const double* const* alpha, const fwi_solve_opts* opts, void* const* data_out,
                      fwi_batch_stats* stats);

/* ------------------------------------------------- building blocks (parity) */
/* y = A_l x for B vectors (Eq. 5 discretised): y_b = x_b - k_l^2 sum W m x_b.
 * precision FWI_FP64: x, y complex128; FWI_FP32_REFINE: complex64 (one FP32
 * operator application). m [n] complex128; freq_index host [B] in [0, nf). */
int fwi_apply_operator(fwi_ctx* ctx, const fwi_problem* prob, int precision, const void* m, int B,
                       const int* freq_index, const void* x, void* y);

/* fwi_apply_operator that allocates nothing, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): its scratch (the frequency
 * indices, the contrast in the working precision and the pass
 * intermediates, about (2 B + 1) n complex values in 2D and (6 B + 1) n in
 * 3D) lives in a static 64 MiB device array of the library, one per GPU,
 * held until the process ends. Same
 * arguments and result as fwi_apply_operator (bit for bit). Requires that
 * the context already holds this problem's Green spectra (any earlier entry
 * point on the problem, e.g. fwi_green_spectrum, builds them; otherwise
 * FWI_E_INVAL); a call needing more scratch than 64 MiB returns FWI_E_NOMEM
 * and writes nothing. Every call on a GPU shares that GPU's scratch: calls
 * that overlap on one GPU (from several contexts or streams) race. */
int fwi_apply_operator_noalloc(fwi_ctx* ctx, const fwi_problem* prob, int precision, const void* m, int B,
                               const int* freq_index, const void* x, void* y);

/* Solve A_l x_b = rhs_b for B right-hand sides with the batched solver.
 * m [n], rhs [B][n], x_out [B][n]: complex128; freq_index host [B]. */
int fwi_solve(fwi_ctx* ctx, const fwi_problem* prob, const void* m, int B, const int* freq_index, const void* rhs,
              const fwi_solve_opts* opts, void* x_out, fwi_stats* stats);

/* Incident fields p0 [ne][n] complex128 of frequency freq_index (Sec. II). */
int fwi_incident(fwi_ctx* ctx, const fwi_problem* prob, int freq_index, void* out);

/* Green spectrum FFT(k^2 W)/npad on the padded grid [Lz][Ly][Lx] complex128. */
int fwi_green_spectrum(fwi_ctx* ctx, const fwi_problem* prob, int freq_index, void* out);

/* Zero-padded forward FFT of in [nz][ny][nx] into out [Lz][Ly][Lx] (precision
 * as in fwi_apply_operator). Diagnostic of the FFT passes. */
int fwi_fft_padded(fwi_ctx* ctx, const fwi_problem* prob, int precision, const void* in, void* out);

/* Jacobian products from stored fields [nf][ne][n] complex128 (Eq. 16-17):
 * out_data [nf][ne][ne] = J a for a [n];  out_m [n] = J^H b for b [nf][ne][ne]. */
int fwi_jacobian_apply(fwi_ctx* ctx, const fwi_problem* prob, const void* fields, const void* a, void* out_data);
int fwi_jacobian_adjoint_apply(fwi_ctx* ctx, const fwi_problem* prob, const void* fields, const void* b,
                               void* out_m);
/* The same products with separate transmit fields and receiver fields (the
 * sensitivity of Sec. IV-B): (J a)_{l,t,j} = k_l^2 dV sum_n p_lt(x_n)
 * p~_lj(x_n) a_n, and its adjoint. tx_fields [nf][nt][n] (e.g. fields_out of
 * fwi_forward_tx), rx_fields [nf][ne][n] (sources at the receivers: fields_out
 * of fwi_forward, which a caller may keep over several model updates, the
 * Born reuse of Sec. IV-B), a [n], out_data [nf][nt][ne], b [nf][nt][ne],
 * out [n]: complex128; 1 <= nt <= ne. */
int fwi_jacobian_apply_tx(fwi_ctx* ctx, const fwi_problem* prob, int nt, const void* tx_fields,
                          const void* rx_fields, const void* a, void* out_data);
int fwi_jacobian_adjoint_apply_tx(fwi_ctx* ctx, const fwi_problem* prob, int nt, const void* tx_fields,
                                  const void* rx_fields, const void* b, void* out);

/* Gauss-Legendre nodes x[q] and weights w[q] on [-1, 1] (1 <= q <= 16) of the
 * element-aperture rule, computed on the host as the kernels receive them;
 * returns 0, or FWI_E_INVAL for q out of range. */
int fwi_host_gauss_legendre(int q, double* x, double* w);

/* ----------------------------------------------------------- measurement */
/* Kernel classes: 0 row forward FFT pass, 1 Green convolution pass (forward
 * FFT, spectrum product, inverse FFT along the depth axis), 2 row inverse
 * pass with epilogue, 3 / 4 forward / inverse elevation passes (3D),
 * 5 Arnoldi inner products (when not fused into the row inverse pass),
 * 6 Arnoldi orthogonalisation alone (after the last step of a cycle),
 * 7 Arnoldi orthogonalisation fused with the row forward pass of the next
 * matvec. */
#define FWI_KC_ROW_FWD 0
#define FWI_KC_CONV 1
#define FWI_KC_ROW_INV 2
#define FWI_KC_Y_FWD 3
#define FWI_KC_Y_INV 4
#define FWI_KC_DOTS 5
#define FWI_KC_ORTH 6
#define FWI_KC_ORTH_FWD 7
/* Class k + 8 is the complex128 launch of class k (k + 0: complex64).
 * Time every launch of the classes in `mask` (bit k = class k) with HIP events
 * that the kernel launch itself records on the context's stream (no extra
 * stream packets); resets the accumulated figures. 0 turns it off. */
int fwi_profile(fwi_ctx* ctx, unsigned mask);
/* Accumulated event time [ms], launch count and algorithmic HBM bytes (the
 * bytes each launch must read and write for the RHS it processes) of a class. */
int fwi_profile_read(const fwi_ctx* ctx, int cls, double* total_ms, long long* launches, double* bytes);

/* ------------------------------------------------------------- autotuner */
/* Each FFT pass of the operator exists in three tile variants (row passes:
 * 2048 / 4096 / 8192 points per workgroup; strided passes: 8 columns x 256
 * threads, 16 x 256, 16 x 512 per workgroup, columns halved while a tile needs
 * more than 80 KiB of LDS). fwi_autotune times every
 * variant of every pass on the device for this problem's grid with B
 * right-hand sides (reps launches each, HIP events) and stores the fastest per
 * (pass, precision, padded length) in the context; a variant replaces the
 * built-in default only if it is at least 2% faster. Later calls use the
 * table. Report rows: 0 row forward, 1 convolution, 2 row inverse, 3 / 4
 * elevation forward / inverse (3D, tuned on their summed time). */
typedef struct fwi_tune_report {
  double variant_ms[5][3];  /* mean time per launch of each variant [ms] */
  int variant[5];           /* chosen variant */
  int default_variant[5];   /* built-in variant before tuning */
} fwi_tune_report;
int fwi_autotune(fwi_ctx* ctx, const fwi_problem* prob, int precision, int B, int reps, fwi_tune_report* report);

/* Batch shape, restart length and inner tolerance of the gradient step (the
 * solver options that set how much work each launch of the Arnoldi kernels
 * carries and how many launches and refinement cycles a solve takes): for
 * every combination of candidate batch caps max_rhs[i] (as
 * fwi_solve_opts.max_rhs; 0 = all frequencies in one batch), restart lengths
 * restart[j] (8, 16 or 32) and inner tolerances inner_rtol[h] (as
 * fwi_solve_opts.inner_rtol, in (0, 1); NULL: base's own, n_inner ignored),
 * with every other option taken from `base`, runs fwi_adjoint_gradient once
 * untimed and then `reps` times, and reports the host wall time of the
 * fastest call (each call synchronises its stream) and the fastest
 * combination. The inner tolerance only acts under FWI_FP32_REFINE: a tighter
 * one costs complex64 iterations and can save a refinement cycle (an FP64
 * operator application); the converged result meets rtol either way. c,
 * alpha, d_obs as in fwi_adjoint_gradient; the gradient itself is discarded.
 * The caller lists only the caps whose memory it accepts (a larger batch
 * keeps more fields and Krylov vectors resident). Runs on the context's
 * current workspace (a caller workspace must fit the largest candidate; the
 * library's own one is released at the end if the search grew it); the FFT
 * tile table and every other context setting are left as they were. A
 * candidate whose solves end unconverged is timed but never chosen
 * (FWI_E_NOCONV when none converges).
 * Errors: FWI_E_INVAL for NULL arguments, reps < 1, counts outside 1..8 caps,
 * 1..3 restarts and 1..3 inner tolerances, a negative cap, a restart other
 * than 8/16/32 or an inner tolerance outside (0, 1); any error of
 * fwi_adjoint_gradient (the first one ends the search). */
typedef struct fwi_solver_tune_report {
  int max_rhs;          /* chosen */
  int restart;          /* chosen */
  double inner_rtol;    /* chosen */
  double ms[3][8][3];   /* [h][i][j] best time of (inner_rtol[h], max_rhs[i], restart[j]) */
} fwi_solver_tune_report;
int fwi_autotune_solver(fwi_ctx* ctx, const fwi_problem* prob, const double* c, const double* alpha,
                        const void* d_obs, const fwi_solve_opts* base, const int* max_rhs, int n_max_rhs,
                        const int* restart, int n_restart, const double* inner_rtol, int n_inner, int reps,
                        fwi_solver_tune_report* report);
/* Copy the tuning table out / in (count = 4*2*11 bytes, -1 = built-in default);
 * in = NULL restores the defaults. For caching tuning results across runs. */
int fwi_get_tuning(const fwi_ctx* ctx, signed char* out, int count);
int fwi_set_tuning(fwi_ctx* ctx, const signed char* in, int count);

/* Host evaluation of the FP64 Bessel routine used by the kernels:
 * out4 = {J0(x), J1(x), Y0(x), Y1(x)} for x > 0. */
void fwi_host_bessel01(double x, double* out4);

#ifdef __cplusplus
}
#endif

#endif /* FWI_H */

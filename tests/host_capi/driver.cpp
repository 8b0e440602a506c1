// Drives the library's C ABI, built for the host against the HIP stand-in,
// through the call sequences of the GPU tests: uneven batches (forward and
// gradient, both precisions, back to back, with waves forced by a small
// memory budget) followed by the eager per-problem entry points, plus one call
// of every other entry point. Run under the address and undefined-behaviour
// sanitizers; prints the emulator's counters and exits non-zero on any error
// code, capture violation or sanitizer report.
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "emu.hpp"
#include "fwi.h"

namespace {

int g_fail = 0;

void check(int rc, const char* what, fwi_ctx* c, bool allow_noconv = false) {
  if (rc == FWI_OK || (allow_noconv && rc == FWI_E_NOCONV)) return;
  std::fprintf(stderr, "[driver] %s failed: rc %d (%s)\n", what, rc, c ? fwi_last_error(c) : "");
  g_fail = 1;
}

// Problem metadata; the frequency and element arrays stay allocated for the
// whole run (problems are copied around with their pointers).
struct Prob {
  fwi_problem p{};
  std::vector<double>* freqs = new std::vector<double>();
  std::vector<double>* elems = new std::vector<double>();
  long n = 0;
};

// A problem as the test recipes make them: cell size 0.154 mm, elements on
// the top face at 0.3 mm pitch (compressed when the aperture would exceed 90%
// of the width), frequencies spread over 0.3-1.0 MHz.
Prob make(int dim, int nx, int ny, int nz, int ne, int nf) {
  Prob q;
  q.p.dim = dim;
  q.p.nx = nx;
  q.p.ny = dim == 3 ? ny : 1;
  q.p.nz = nz;
  q.p.dx = 0.154e-3;
  q.p.c0 = 1540.0;
  q.p.nf = nf;
  for (int l = 0; l < nf; ++l) q.freqs->push_back(nf > 1 ? 0.3e6 + 0.7e6 * l / (nf - 1) : 0.9e6);
  const double wx = nx * q.p.dx;
  double pitch = 0.3e-3;
  if (pitch * (ne - 1) > 0.9 * wx) pitch = 0.9 * wx / ne;
  for (int e = 0; e < ne; ++e) {
    q.elems->push_back(wx / 2 + (e - (ne - 1) / 2.0) * pitch);
    q.elems->push_back(dim == 3 ? q.p.ny * q.p.dx / 2 : 0.0);
    q.elems->push_back(0.0);
  }
  q.p.ne = ne;
  q.p.freq_hz = q.freqs->data();
  q.p.elem_xyz = q.elems->data();
  q.n = (long)nx * q.p.ny * nz;
  return q;
}

template <typename T>
T* dev(size_t count, double fill = 0.0) {
  T* p = static_cast<T*>(std::malloc(sizeof(T) * (count ? count : 1)));
  for (size_t i = 0; i < count; ++i) p[i] = T(fill);
  return p;
}

fwi_solve_opts opts(int prec, int restart) {
  fwi_solve_opts o;
  fwi_default_opts(&o);
  o.precision = prec;
  o.rtol = 1e-12;
  o.restart = restart;
  o.inner_rtol = 1e-3;
  return o;
}

struct Inst {
  Prob q;
  double *c, *alpha;
  std::complex<double>* dobs;
  std::complex<double>* grad;
  std::complex<double>* data;
};

Inst inst(int nx, int nz, int ne, int nf) {
  Inst I;
  I.q = make(2, nx, 1, nz, ne, nf);
  I.c = dev<double>(I.q.n, 1540.0);
  for (long i = 0; i < I.q.n; i += 7) I.c[i] = 1500.0;
  I.alpha = dev<double>(I.q.n, 0.0);
  I.dobs = dev<std::complex<double>>((size_t)nf * ne * ne, 0.25);
  I.grad = dev<std::complex<double>>(I.q.n);
  I.data = dev<std::complex<double>>((size_t)nf * ne * ne);
  return I;
}

void run_batch(fwi_ctx* ctx, std::vector<Inst>& insts, int prec, int restart, bool gradient) {
  std::vector<fwi_problem> probs;
  std::vector<const double*> cs, as;
  std::vector<const void*> ds;
  std::vector<void*> gs, outs;
  for (Inst& I : insts) {
    probs.push_back(I.q.p);
    cs.push_back(I.c);
    as.push_back(I.alpha);
    ds.push_back(I.dobs);
    gs.push_back(I.grad);
    outs.push_back(I.data);
  }
  fwi_solve_opts o = opts(prec, restart);
  fwi_batch_stats st{};
  if (gradient) {
    std::vector<double> mis(insts.size());
    check(fwi_adjoint_gradient_batch(ctx, (int)insts.size(), probs.data(), cs.data(), as.data(), ds.data(), &o,
                                     mis.data(), gs.data(), &st),
          "fwi_adjoint_gradient_batch", ctx);
  } else {
    check(fwi_forward_batch(ctx, (int)insts.size(), probs.data(), cs.data(), as.data(), &o, outs.data(), &st),
          "fwi_forward_batch", ctx);
  }
  std::printf("[driver] batch %s prec %d restart %d: waves %d, graph launches %d, iterations %d, solves %lld\n",
              gradient ? "gradient" : "forward", prec, restart, st.waves, st.graph_launches, st.iterations,
              st.solves);
}

void run_eager_gradient(fwi_ctx* ctx, Inst& I, int prec, int restart) {
  fwi_solve_opts o = opts(prec, restart);
  double phi = 0.0;
  fwi_stats st{};
  std::vector<double> gc(I.q.n), ga(I.q.n);
  double* dgc = dev<double>(I.q.n);
  double* dga = dev<double>(I.q.n);
  check(fwi_adjoint_gradient(ctx, &I.q.p, I.c, I.alpha, I.dobs, &o, &phi, I.grad, dgc, dga, &st),
        "fwi_adjoint_gradient", ctx);
  std::free(dgc);
  std::free(dga);
}

void every_entry(fwi_ctx* ctx, int dim, bool planes = false) {
  // planes: a 3D grid whose padded lateral and elevation lengths (128) take
  // the fused lateral-elevation passes of the complex64 operator
  Prob q = dim == 2 ? make(2, 24, 1, 20, 4, 2) : planes ? make(3, 60, 58, 6, 3, 2) : make(3, 10, 8, 9, 3, 2);
  const long n = q.n;
  const int ne = q.p.ne, nf = q.p.nf;
  double* c = dev<double>(n, 1540.0);
  double* a = dev<double>(n, 0.0);
  auto* data = dev<std::complex<double>>((size_t)nf * ne * ne);
  auto* fields = dev<std::complex<double>>((size_t)nf * ne * n);
  auto* dobs = dev<std::complex<double>>((size_t)nf * ne * ne, 0.5);
  auto* gm = dev<std::complex<double>>(n);
  for (int prec = 0; prec < 2; ++prec) {
    fwi_solve_opts o = opts(prec, 8);
    fwi_stats st{};
    check(fwi_forward(ctx, &q.p, c, a, &o, data, fields, &st), "fwi_forward", ctx);
    double phi;
    check(fwi_adjoint_gradient(ctx, &q.p, c, a, dobs, &o, &phi, gm, nullptr, nullptr, &st), "gradient", ctx);
    o.max_rhs = ne;  // one frequency per batch
    check(fwi_adjoint_gradient(ctx, &q.p, c, a, dobs, &o, &phi, gm, nullptr, nullptr, &st), "gradient grouped", ctx);
    o.max_rhs = 0;
    o.reciprocity_adjoint = 1;
    check(fwi_adjoint_gradient(ctx, &q.p, c, a, dobs, &o, &phi, gm, nullptr, nullptr, &st), "gradient recip", ctx);
    o.reciprocity_adjoint = 0;
    check(fwi_vjp(ctx, &q.p, gm, dobs, &o, gm, &st), "vjp", ctx);
    check(fwi_vjp_fields(ctx, &q.p, gm, fields, dobs, &o, gm, &st), "vjp_fields", ctx);
    {
      // transmit chunks (ragged last chunk) and complex64 field output
      fwi_solve_opts oc = o;
      oc.tx_chunk = ne - 1;
      oc.fields_c64 = 1;
      check(fwi_forward(ctx, &q.p, c, a, &oc, data, fields, &st), "forward chunked c64 fields", ctx);
      oc.fields_c64 = 0;
      check(fwi_forward(ctx, &q.p, c, a, &oc, data, fields, &st), "forward chunked", ctx);
      check(fwi_adjoint_gradient(ctx, &q.p, c, a, dobs, &oc, &phi, gm, nullptr, nullptr, &st), "gradient chunked",
            ctx);
      check(fwi_vjp(ctx, &q.p, gm, dobs, &oc, gm, &st), "vjp chunked", ctx);
      check(fwi_vjp_fields(ctx, &q.p, gm, fields, dobs, &oc, gm, &st), "vjp_fields chunked", ctx);
      oc.reciprocity_adjoint = 1;
      if (fwi_adjoint_gradient(ctx, &q.p, c, a, dobs, &oc, &phi, gm, nullptr, nullptr, &st) != FWI_E_UNSUPPORTED) {
        std::fprintf(stderr, "[driver] reciprocity with transmit chunks not refused\n");
        g_fail = 1;
      }
    }
    // synthesised transmits
    const int nt = 2;
    auto* w = dev<std::complex<double>>((size_t)nf * nt * ne, 1.0);
    auto* dtx = dev<std::complex<double>>((size_t)nf * nt * ne);
    auto* ftx = dev<std::complex<double>>((size_t)nf * nt * n);
    check(fwi_forward_tx(ctx, &q.p, c, a, nt, w, &o, dtx, ftx, &st), "forward_tx", ctx);
    check(fwi_adjoint_gradient_tx(ctx, &q.p, c, a, nt, w, dtx, &o, &phi, gm, nullptr, nullptr, &st), "gradient_tx",
          ctx);
    {
      fwi_solve_opts oc = o;
      oc.tx_chunk = 1;
      oc.fields_c64 = 1;
      check(fwi_forward_tx(ctx, &q.p, c, a, nt, w, &oc, dtx, ftx, &st), "forward_tx chunked c64", ctx);
      check(fwi_adjoint_gradient_tx(ctx, &q.p, c, a, nt, w, dtx, &oc, &phi, gm, nullptr, nullptr, &st),
            "gradient_tx chunked", ctx);
    }
    check(fwi_jacobian_apply_tx(ctx, &q.p, nt, ftx, fields, gm, dtx), "jacobian_apply_tx", ctx);
    check(fwi_jacobian_adjoint_apply_tx(ctx, &q.p, nt, ftx, fields, dtx, gm), "jacobian_adjoint_apply_tx", ctx);
    check(fwi_jacobian_apply(ctx, &q.p, fields, gm, data), "jacobian_apply", ctx);
    check(fwi_jacobian_adjoint_apply(ctx, &q.p, fields, data, gm), "jacobian_adjoint_apply", ctx);
    // ADMM on the forward mesh and on a 2x coarser mesh, element and synthesised transmits
    for (int r = 1; r <= 2; ++r) {
      const long nc = (long)((q.p.nx + r - 1) / r) * (dim == 3 ? (q.p.ny + r - 1) / r : 1) * ((q.p.nz + r - 1) / r);
      auto* m = dev<std::complex<double>>(nc, 0.01);
      auto* g = dev<std::complex<double>>((size_t)dim * nc);
      auto* u = dev<std::complex<double>>((size_t)dim * nc);
      auto* mref = dev<std::complex<double>>(nc);
      fwi_admm_params prm{1e-3, 1e-2, 1e-5, 3, 0.0, 1e-2, r};
      fwi_admm_report rep{};
      check(fwi_tv_admm_step(ctx, &q.p, &prm, m, g, u, mref, dobs, &o, &rep, &st), "admm", ctx);
      check(fwi_tv_admm_step_tx(ctx, &q.p, &prm, nt, w, fields, 1, m, g, u, nullptr, dtx, &o, &rep, &st), "admm_tx",
            ctx);
      std::vector<double> hist(3);
      int done = 0;
      check(fwi_invert(ctx, &q.p, &prm, 3, 0.0, 0, nullptr, nullptr, 0, m, g, u, mref, dobs, &o, hist.data(), &done,
                       &st),
            "invert", ctx);
      check(fwi_invert(ctx, &q.p, &prm, 3, 0.0, nt, w, fields, 2, m, g, u, mref, dtx, &o, hist.data(), &done, &st),
            "invert_tx", ctx);
      std::free(m);
      std::free(g);
      std::free(u);
      std::free(mref);
    }
    std::free(w);
    std::free(dtx);
    std::free(ftx);
    // building blocks
    std::vector<int> fi = {0, nf - 1, 0};
    const size_t es = prec ? 8 : 16;
    void* x = std::calloc(3 * n, es);
    void* y = std::calloc(3 * n, es);
    check(fwi_apply_operator(ctx, &q.p, prec, gm, 3, fi.data(), x, y), "apply_operator", ctx);
    check(fwi_apply_operator_noalloc(ctx, &q.p, prec, gm, 3, fi.data(), x, y), "apply_operator_noalloc", ctx);
    check(fwi_apply_operator_noalloc(ctx, &q.p, prec, gm, 1, fi.data(), x, y), "apply_operator_noalloc", ctx);
    auto* rhs = dev<std::complex<double>>(3 * n, 1.0);
    auto* xs = dev<std::complex<double>>(3 * n);
    check(fwi_solve(ctx, &q.p, gm, 3, fi.data(), rhs, &o, xs, &st), "solve", ctx);
    check(fwi_incident(ctx, &q.p, nf - 1, fields), "incident", ctx);
    int pad[3];
    pad[0] = fwi_padded_length(q.p.nx);
    pad[1] = dim == 3 ? fwi_padded_length(q.p.ny) : 1;
    pad[2] = fwi_padded_length(q.p.nz);
    auto* spec = dev<std::complex<double>>((size_t)pad[0] * pad[1] * pad[2]);
    check(fwi_green_spectrum(ctx, &q.p, nf - 1, spec), "green_spectrum", ctx);
    check(fwi_fft_padded(ctx, &q.p, prec, x, spec), "fft_padded", ctx);
    fwi_tune_report rep{};
    check(fwi_autotune(ctx, &q.p, prec, 5, 1, &rep), "autotune", ctx);
    {
      // batch caps of whole frequencies, one frequency and the whole problem; two restart lengths
      const int mr[3] = {0, ne, 2 * ne};
      const int rs[2] = {8, 16};
      fwi_solver_tune_report srep{};
      fwi_solve_opts ot = opts(prec, 8);
      const double ir[2] = {1e-3, 1e-4};
      check(fwi_autotune_solver(ctx, &q.p, c, a, dobs, &ot, mr, 3, rs, 2, ir, 2, 1, &srep), "autotune_solver", ctx);
      if ((srep.restart != 8 && srep.restart != 16) || (srep.inner_rtol != ir[0] && srep.inner_rtol != ir[1])) {
        std::fprintf(stderr, "[driver] autotune_solver chose restart %d, inner %g\n", srep.restart, srep.inner_rtol);
        g_fail = 1;
      }
      check(fwi_autotune_solver(ctx, &q.p, c, a, dobs, &ot, mr, 1, rs, 1, nullptr, 0, 1, &srep), "autotune_solver",
            ctx);
      if (srep.inner_rtol != ot.inner_rtol) {
        std::fprintf(stderr, "[driver] autotune_solver without inner candidates chose %g\n", srep.inner_rtol);
        g_fail = 1;
      }
      const int bad[1] = {-1};
      if (fwi_autotune_solver(ctx, &q.p, c, a, dobs, &ot, bad, 1, rs, 2, nullptr, 0, 1, &srep) != FWI_E_INVAL) {
        std::fprintf(stderr, "[driver] negative batch cap not refused\n");
        g_fail = 1;
      }
      const double bad_ir[1] = {2.0};
      if (fwi_autotune_solver(ctx, &q.p, c, a, dobs, &ot, mr, 1, rs, 1, bad_ir, 1, 1, &srep) != FWI_E_INVAL) {
        std::fprintf(stderr, "[driver] inner tolerance above 1 not refused\n");
        g_fail = 1;
      }
    }
    double* co = dev<double>(n);
    check(fwi_sos_from_contrast(ctx, &q.p, gm, co, co), "sos_from_contrast", ctx);
    std::free(co);
    std::free(spec);
    std::free(rhs);
    std::free(xs);
    std::free(x);
    std::free(y);
  }
  // a caller workspace too small: NOMEM, no overrun
  char* ws = static_cast<char*>(std::malloc(4096));
  check(fwi_set_workspace(ctx, ws, 4096), "set_workspace", ctx);
  fwi_solve_opts o = opts(0, 8);
  fwi_stats st{};
  if (fwi_forward(ctx, &q.p, c, a, &o, data, nullptr, &st) != FWI_E_NOMEM) {
    std::fprintf(stderr, "[driver] small caller workspace not refused\n");
    g_fail = 1;
  }
  size_t need = 0;
  check(fwi_workspace_size(&q.p, &o, 0, &need), "workspace_size", ctx);
  char* ws2 = static_cast<char*>(std::malloc(need));
  check(fwi_set_workspace(ctx, ws2, need), "set_workspace", ctx);
  check(fwi_forward(ctx, &q.p, c, a, &o, data, nullptr, &st), "forward in caller workspace", ctx);
  check(fwi_set_workspace(ctx, nullptr, 0), "set_workspace", ctx);
  std::free(ws);
  std::free(ws2);
  std::free(c);
  std::free(a);
  std::free(data);
  std::free(fields);
  std::free(dobs);
  std::free(gm);
}

}  // namespace

int main(int argc, char** argv) {
  const std::string what = argc > 1 ? argv[1] : "all";
  fwi_ctx* ctx = nullptr;
  hipStream_t user = nullptr;
  hipStreamCreateWithFlags(&user, hipStreamNonBlocking);
  check(fwi_create(&ctx, 0, user), "fwi_create", nullptr);
  if (!ctx) return 1;
  if (what == "all" || what == "batch") {
    // the uneven-batch parity sequence: two batch gradients per precision,
    // then the eager gradient of every instance
    std::vector<Inst> small = {inst(24, 20, 4, 2), inst(40, 33, 6, 1), inst(33, 48, 5, 3)};
    for (int prec = 0; prec < 2; ++prec) {
      run_batch(ctx, small, prec, 16, true);
      run_batch(ctx, small, prec, 16, true);
      for (Inst& I : small) run_eager_gradient(ctx, I, prec, 16);
    }
    // the full-size sequence: FP64 forward batch, mixed gradient batch,
    // eager gradients, with memory for a few instances per wave only
    std::vector<Inst> many;
    const int shapes[][4] = {{32, 32, 8, 1}, {48, 48, 12, 2}, {40, 40, 5, 4}, {64, 64, 16, 3}, {32, 32, 6, 2},
                             {48, 48, 9, 1}, {24, 24, 4, 4}, {64, 64, 7, 2}};
    for (auto& s : shapes) many.push_back(inst(s[0], s[1], s[2], s[3]));
    emu::mem_free = size_t(6) << 20;
    run_batch(ctx, many, 0, 16, false);
    run_batch(ctx, many, 1, 16, true);
    for (int k : {0, 3, 7}) run_eager_gradient(ctx, many[k], 1, 16);
    emu::mem_free = size_t(8) << 30;
    run_batch(ctx, many, 1, 8, true);
    run_batch(ctx, many, 1, 32, true);
    for (int k : {1, 6}) run_eager_gradient(ctx, many[k], 0, 32);
  }
  if (what == "all" || what == "entries") {
    every_entry(ctx, 2);
    every_entry(ctx, 3);
    every_entry(ctx, 3, true);
    check(fwi_set_plane_fusion(ctx, 1), "plane fusion on", ctx);
    every_entry(ctx, 3, true);
    check(fwi_set_plane_fusion(ctx, 0), "plane fusion off", ctx);
    if (fwi_set_plane_fusion(ctx, 2) != FWI_E_INVAL) {
      std::fprintf(stderr, "[driver] plane fusion value 2 not refused\n");
      g_fail = 1;
    }
  }
  fwi_destroy(ctx);
  hipStreamDestroy(user);
  const emu::Counts& k = emu::counts();
  std::printf("[driver] kernels live %ld, captured %ld, graph launches %ld, captures %ld, copies captured %ld, "
              "violations %ld\n",
              k.kernels_live, k.kernels_captured, k.graph_launches, k.captures, k.copies_captured, k.violations);
  if (k.violations) g_fail = 1;
  std::printf(g_fail ? "[driver] FAILED\n" : "[driver] OK\n");
  return g_fail;
}

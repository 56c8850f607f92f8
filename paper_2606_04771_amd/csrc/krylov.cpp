// Krylov exponential exp(tau H_eff) x on the device.
//
// The paper evolves each merged block with a Krylov matrix exponential whose
// dimension is chosen adaptively (supplementary section S2.2).  Here: Lanczos
// with two passes of classical Gram-Schmidt against the whole basis (FP64),
// the small tridiagonal exponential on the host, and the a-posteriori
// estimate beta_m |[exp(tau T_m)]_{m,1}| |x| as the stopping rule.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>

#include "device.hpp"
#include "tridiag.hpp"

namespace tdvp {

int copy_blocks(tdvp_ctx* ctx, const Blocks& src, const Blocks& dst, double s) {
  // a grouped-GEMM program made only of direct terms
  Program p;
  for (int j = 0; j < dst.n(); ++j) {
    int i = src.find(dst.k(j));
    DevOut ob{};
    ob.c_off = dst.off[j];
    ob.ldc = ob.M = (int32_t)dst.rows[j];
    ob.N = (int32_t)dst.cols[j];
    ob.t_begin = ob.t_end = ob.d_begin = (int32_t)p.terms.size();
    if (i >= 0) {
      DevTerm d{};
      d.a_buf = 0;
      d.a_off = src.off[i];
      d.lda = (int32_t)src.rows[i];
      d.coef = s;
      p.terms.push_back(d);
    }
    ob.d_end = (int32_t)p.terms.size();
    p.outs.push_back(ob);
  }
  p.finalize();
  int rc = upload(ctx, p);
  if (rc) return rc;
  Bufs b{};
  b.p[0] = (const double*)src.data;
  // the program's arrays return to the stream-ordered pool when p goes out of scope
  return launch_gemm(ctx, p, b, (double*)dst.data, TDVP_FP64);
}

namespace {

bool contiguous(const Blocks& x, int64_t& n) {
  std::vector<std::pair<int64_t, int64_t>> iv;
  for (int i = 0; i < x.n(); ++i) iv.push_back({x.off[i], x.rows[i] * x.cols[i]});
  std::sort(iv.begin(), iv.end());
  int64_t pos = 0;
  for (auto& v : iv) {
    if (v.first != pos) return false;
    pos += v.second;
  }
  n = pos;
  return true;
}

// One Lanczos iteration recorded as a graph: w = op(x), two Gram-Schmidt
// passes against v_0..v_j, |w|^2, the copy of the coefficients to the host,
// and x = v_{j+1} = w / |w|; j is read from and advanced in device memory.
struct IterGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~IterGraph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

}  // namespace

// Lanczos exponential of a device operator on a contiguous vector of n
// complex elements, in place.  The operator writes op(v) to w (both
// contiguous, n elements); flops_per_apply is added to out.heff_flops.
int krylov_core(tdvp_ctx* ctx, int64_t n, double* x, const std::function<int(const double*, double*)>& op,
                double flops_per_apply, std::complex<double> tau, double tol, int maxdim, KrylovResult& out,
                const std::function<bool()>& capturable) {
  out = KrylovResult();
  if (n == 0) return TDVP_OK;
  const int64_t stride = n;
  // basis v_0..v_{maxdim-1} (complex128, or complex64 with the FP32 basis
  // storage), w, and the FP64 operator input Xg: the current basis vector,
  // which the graph reads from a fixed address and which the complex64 basis
  // keeps in full precision (the recurrence itself stays in FP64; only the
  // re-orthogonalisation and the final combination read the rounded copies)
  const bool v32 = ctx->krylov_fp32;
  const bool try_graph = capturable && ctx->graphs && maxdim > 1;
  const bool own_x = try_graph || v32;
  const size_t vbytes = (v32 ? sizeof(float) : sizeof(double)) * 2 * (size_t)stride * maxdim;
  const size_t vpad = (vbytes + 255) & ~(size_t)255;
  TDVP_HIP(ctx, ctx->ws_krylov.ensure(vpad + sizeof(double) * 2 * (size_t)stride * (own_x ? 2 : 1)));
  TDVP_HIP(ctx, ctx->ws_small.ensure(1 << 16));
  if (try_graph) TDVP_HIP(ctx, ctx->ws_lanczos.ensure(lanczos_partial_bytes(n, maxdim)));
  double* V = (double*)ctx->ws_krylov.p;
  double* W = (double*)((char*)ctx->ws_krylov.p + vpad);
  double* Xg = own_x ? W + 2 * stride : nullptr;
  double* d_small = (double*)ctx->ws_small.p;
  double* h_small = (double*)ctx->host_small;
  double* d_c1 = d_small;          // 2*64
  double* d_c2 = d_small + 128;    // 2*64
  double* d_nrm = d_small + 256;   // 2
  double* d_y = d_small + 512;     // 2*64
  int* d_j = (int*)(d_small + 2048);
  IterGraph graph;
  bool replay = false;

  // v0 = x / |x|
  int rc;
  double* x0 = v32 ? Xg : V;   // FP64 copy of v0
  TDVP_HIP(ctx, hipMemcpyAsync(x0, x, sizeof(double) * 2 * n, hipMemcpyDeviceToDevice, ctx->stream));
  if ((rc = vec_norm2(ctx, x0, n, d_nrm))) return rc;
  TDVP_HIP(ctx, hipMemcpyAsync(h_small, d_nrm, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  TDVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (h_small[1] != 0.0 || !std::isfinite(h_small[0]))
    return set_error(ctx, TDVP_E_NONFINITE, "non-finite entries in the Krylov start vector");
  const double nrm = std::sqrt(h_small[0]);
  out.norm = nrm;
  if (nrm == 0.0) {
    out.converged = 1;
    return TDVP_OK;
  }
  if ((rc = vec_scale_copy(ctx, x0, x0, 1.0 / nrm, n))) return rc;
  if (v32 && (rc = vec_store_basis32(ctx, V, x0, n))) return rc;

  std::vector<double> alpha, beta;
  std::vector<std::complex<double>> y;
  for (int j = 0; j < maxdim; ++j) {
    // FP64 operator input of this iteration: the basis slot itself, or Xg
    // (always Xg with the complex64 basis, where it holds v_j in FP64)
    double* vj = v32 ? Xg : V + 2 * stride * j;
    // from the second iteration on (workspaces sized), once the operator can
    // be recorded: capture one iteration and replay it from here on
    if (try_graph && !replay && j >= 1 && capturable()) {
      if ((rc = vec_set_index(ctx, d_j, j))) return rc;
      if (!v32) TDVP_HIP(ctx, hipMemcpyAsync(Xg, vj, sizeof(double) * 2 * n, hipMemcpyDeviceToDevice, ctx->stream));
      bool ok = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
      if (ok) {
        int crc = op(Xg, W);
        if (!crc)
          crc = vec_lanczos_orth_it(ctx, W, V, stride, maxdim, n, d_j, d_c1, d_c2, d_nrm, ctx->ws_lanczos.p, v32);
        if (!crc && hipMemcpyAsync(h_small, d_small, 258 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream) !=
                        hipSuccess)
          crc = TDVP_E_HIP;
        if (!crc) crc = vec_lanczos_advance_it(ctx, V, stride, Xg, W, n, d_nrm, d_j, maxdim, v32);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(ctx->stream, &g);
        graph.graph = g;
        ok = !crc && e == hipSuccess && g &&
             hipGraphInstantiate(&graph.exec, g, nullptr, nullptr, 0) == hipSuccess;
      }
      if (!ok) {   // stay with direct launches
        (void)hipGetLastError();
        if (ctx->verbose) std::fprintf(stderr, "[tdvp]   Lanczos graph capture failed; direct launches\n");
      }
      replay = ok;
      if (!ok) {   // the capture may have left launches unrecorded: start the iteration afresh
        TDVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
      }
    }
    if (replay) {
      TDVP_HIP(ctx, hipGraphLaunch(graph.exec, ctx->stream));
      out.heff_flops += flops_per_apply;
      ++out.graph_iters;
    } else {
      if ((rc = op(vj, W))) return rc;
      out.heff_flops += flops_per_apply;
      // two passes of classical Gram-Schmidt against v_0..v_j
      if ((rc = vec_dots(ctx, V, stride, j + 1, W, n, d_c1, v32))) return rc;
      if ((rc = vec_subtract_combo(ctx, W, V, stride, j + 1, d_c1, n, nullptr, v32))) return rc;
      if ((rc = vec_dots(ctx, V, stride, j + 1, W, n, d_c2, v32))) return rc;
      if ((rc = vec_subtract_combo(ctx, W, V, stride, j + 1, d_c2, n, d_nrm, v32))) return rc;
      TDVP_HIP(ctx, hipMemcpyAsync(h_small, d_small, 258 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    }
    TDVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    double a = h_small[2 * j] + h_small[128 + 2 * j];
    double b2 = h_small[256];
    if (!std::isfinite(a) || !std::isfinite(b2))
      return set_error(ctx, TDVP_E_NONFINITE, "non-finite Lanczos coefficient");
    double b = std::sqrt(std::max(b2, 0.0));
    alpha.push_back(a);
    if (!tridiag_expm_e1(alpha, beta, tau, nrm, y))
      return set_error(ctx, TDVP_E_NOCONV, "tridiagonal eigensolver did not converge");
    double err = b * std::abs(y[j]);
    bool breakdown = b < 1e-14 * 1.0;   // basis vectors have unit norm
    bool done = breakdown || err <= tol * nrm || j + 1 == maxdim;
    out.iters = j + 1;
    out.err = err;
    if (done) {
      out.converged = (breakdown || err <= tol * nrm) ? 1 : 0;
      out.alpha = alpha;
      out.beta = beta;
      out.beta.push_back(b);
      for (int k = 0; k <= j; ++k) {
        h_small[512 + 2 * k] = y[k].real();
        h_small[512 + 2 * k + 1] = y[k].imag();
      }
      TDVP_HIP(ctx, hipMemcpyAsync(d_y, h_small + 512, sizeof(double) * 2 * (j + 1), hipMemcpyHostToDevice,
                                   ctx->stream));
      if ((rc = vec_combo(ctx, x, V, stride, j + 1, d_y, n, v32))) return rc;
      TDVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
      if (!out.converged) return set_error(ctx, TDVP_E_NOCONV, "Krylov tolerance not reached within maxdim");
      return TDVP_OK;
    }
    beta.push_back(b);
    if (!replay) {   // v_{j+1} = w / |w| by the replayed iteration's own kernel (same rounding)
      double* vn = v32 ? Xg : V + 2 * stride * (j + 1);
      if ((rc = vec_set_index(ctx, d_j, j))) return rc;
      if ((rc = vec_lanczos_advance_it(ctx, V, stride, vn, W, n, d_nrm, d_j, maxdim, v32))) return rc;
    }
  }
  return TDVP_OK;
}

int krylov_dev(tdvp_ctx* ctx, const tdvp_model& m, int site, int nsites, const HeffInputs& in_user,
               std::complex<double> tau, double tol, int maxdim, KrylovResult& out) {
  out = KrylovResult();
  int64_t n = 0;
  HeffInputs in = in_user;
  bool compact = contiguous(in.x, n);
  if (!compact) {
    // Lanczos vectors use a compact copy of the block layout
    Blocks xc;
    xc.keylen = in.x.keylen;
    int64_t o = 0;
    for (int i = 0; i < in.x.n(); ++i) {
      xc.push(in.x.k(i), o, in.x.rows[i], in.x.cols[i]);
      o += in.x.rows[i] * in.x.cols[i];
    }
    xc.size = o;
    in.x = xc;
    n = o;
  }
  if (n == 0) return TDVP_OK;
  int rc;
  Blocks yb = in.x;   // output layout of the apply = compact layout
  auto prog = heff_program(ctx, m, site, nsites, in, yb, rc);
  if (rc) return rc;
  Bufs bufs{};
  bufs.p[1] = (const double*)in.Le.data;
  bufs.p[2] = (const double*)in.Re.data;
  auto op = [&](const double* v, double* w) -> int {
    bufs.p[0] = v;
    return launch_gemm(ctx, *prog, bufs, w, ctx->precision);
  };
  // recordable once the tiling autotuner (events, host reads) has decided
  auto capturable = [&]() { return ctx->precision != TDVP_FP64 || !prog->tuning(); };
  double* xd = (double*)in_user.x.data;
  if (!compact) {
    // work on a compact copy (after the Krylov basis in the scratch area)
    TDVP_HIP(ctx, ctx->ws_compact.ensure(sizeof(double) * 2 * (size_t)n));
    Blocks xc = in.x;
    xc.data = ctx->ws_compact.p;
    if ((rc = copy_blocks(ctx, in_user.x, xc, 1.0))) return rc;
    xd = (double*)ctx->ws_compact.p;
  }
  rc = krylov_core(ctx, n, xd, op, prog->flops, tau, tol, maxdim, out, capturable);
  if (rc && rc != TDVP_E_NOCONV) return rc;
  if (!compact) {
    Blocks xc = in.x;
    xc.data = ctx->ws_compact.p;
    int rc2 = copy_blocks(ctx, xc, in_user.x, 1.0);
    if (rc2) return rc2;
    TDVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  }
  return rc;
}

}  // namespace tdvp

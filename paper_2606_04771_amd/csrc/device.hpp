// Device-side building blocks shared by the C-ABI entry points.
#pragma once

#include <complex>
#include <functional>
#include <memory>
#include <vector>

#include "common.hpp"
#include "ctx.hpp"

namespace tdvp {

std::shared_ptr<Program> heff_program(tdvp_ctx* ctx, const tdvp_model& m, int site, int nsites,
                                      const HeffInputs& in, const Blocks& y, int& rc);

// Environment update on the device (programs cached by structure).
int env_update_dev(tdvp_ctx* ctx, const tdvp_model& m, int site, int dir, const EnvInputs& in,
                   double* flops = nullptr);

// The two grouped-GEMM stages of an environment update; scratch = complex
// elements of the stage-1 products.
struct EnvPrograms {
  std::shared_ptr<Program> s1, s2;
  int64_t scratch = 0;
};
// Uploaded and cached (device memory from the context's allocator).
EnvPrograms env_programs(tdvp_ctx* ctx, const tdvp_model& m, int site, int dir, const EnvInputs& in, int& rc);
// Host description only (cached on the host; no device memory touched).
EnvPrograms env_programs_host(tdvp_ctx* ctx, const tdvp_model& m, int site, int dir, const EnvInputs& in);

// Address of the static scratch on the current device (taken once per device
// by the first context created there).  Errors: HIP.
int noalloc_init(tdvp_ctx* ctx);

struct KrylovResult {
  int iters = 0;
  int converged = 0;
  double err = 0.0, norm = 0.0;
  std::vector<double> alpha, beta;
  double heff_flops = 0.0;
  int graph_iters = 0;   // iterations replayed from the captured graph
};
// x <- exp(tau H_eff) x (x = in.x, data in place).
int krylov_dev(tdvp_ctx* ctx, const tdvp_model& m, int site, int nsites, const HeffInputs& in,
               std::complex<double> tau, double tol, int maxdim, KrylovResult& out);

// x <- exp(tau op) x for a device operator on n contiguous complex elements.
// capturable(), when given, says whether op may now be recorded into a graph
// (no allocation, synchronisation or measurement inside); from then on one
// captured Lanczos iteration is replayed for every further iteration.
int krylov_core(tdvp_ctx* ctx, int64_t n, double* x, const std::function<int(const double*, double*)>& op,
                double flops_per_apply, std::complex<double> tau, double tol, int maxdim, KrylovResult& out,
                const std::function<bool()>& capturable = {});

// Copy blocks: dst[j] = src[i] for blocks with equal keys (scaled by s).
int copy_blocks(tdvp_ctx* ctx, const Blocks& src, const Blocks& dst, double s);

}  // namespace tdvp

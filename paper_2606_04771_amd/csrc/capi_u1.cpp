// C-ABI entry points of the abelian U(1) x U(1) variant: layouts and plans
// (host), effective-Hamiltonian apply, Krylov exponential and environment
// update (device), on the same grouped-GEMM programs and Lanczos kernels as
// the U(1) x SU(2) calls.
#include <hip/hip_runtime.h>

#include <complex>
#include <cstring>
#include <string>

#include "common.hpp"
#include "ctx.hpp"
#include "device.hpp"
#include "plan.hpp"

using namespace tdvp;

extern "C" {

int tdvp_u1_center_layout(const tdvp_bond* left, const tdvp_bond* right, int32_t nsites, int32_t* nblocks,
                          int32_t* keys, int64_t* offsets, int64_t* total) {
  return guarded(nullptr, [&]() -> int {
    std::string err;
    if (nsites != 1 && nsites != 2) return set_error(nullptr, TDVP_E_INVALID, "nsites must be 1 or 2");
    if (!nblocks) return set_error(nullptr, TDVP_E_INVALID, "nblocks is null");
    Bond l, r;
    int rc = u1_load_bond(l, left, err);
    if (!rc) rc = u1_load_bond(r, right, err);
    if (rc) return set_error(nullptr, rc, err);
    Blocks b;
    u1_layout_center(l, r, nsites, b);
    *nblocks = b.n();
    if (total) *total = b.size;
    if (keys) std::memcpy(keys, b.key.data(), sizeof(int) * b.key.size());
    if (offsets) std::memcpy(offsets, b.off.data(), sizeof(int64_t) * b.off.size());
    return TDVP_OK;
  });
}

int tdvp_u1_env_layout(const tdvp_bond* bond, int32_t* nblocks, int32_t* keys, int64_t* offsets, int64_t* total) {
  return guarded(nullptr, [&]() -> int {
    std::string err;
    if (!nblocks) return set_error(nullptr, TDVP_E_INVALID, "nblocks is null");
    Bond b;
    int rc = u1_load_bond(b, bond, err);
    if (rc) return set_error(nullptr, rc, err);
    Blocks e;
    u1_layout_env(b, e);
    *nblocks = e.n();
    if (total) *total = e.size;
    if (keys) std::memcpy(keys, e.key.data(), sizeof(int) * e.key.size());
    if (offsets) std::memcpy(offsets, e.off.data(), sizeof(int64_t) * e.off.size());
    return TDVP_OK;
  });
}

int tdvp_u1_heff_plan(const tdvp_model* model, int32_t site, int32_t nsites, const tdvp_bond* left,
                      const tdvp_bond* right, const tdvp_blocks* Lenv, const tdvp_blocks* Renv, const tdvp_blocks* x,
                      int64_t* nterms, tdvp_term* terms, double* flops) {
  return guarded(nullptr, [&]() -> int {
    HeffInputs in;
    std::string err;
    int rc = u1_load_heff_inputs(in, model, site, nsites, left, right, Lenv, Renv, x, err);
    if (rc) return set_error(nullptr, rc, err);
    if (!nterms) return set_error(nullptr, TDVP_E_INVALID, "nterms is null");
    std::vector<HTerm> t;
    double f = 0;
    u1_plan_heff(*model, site, nsites, in.l, in.r, in.Le, in.Re, in.x, t, f);
    if (terms) {
      const int64_t n = std::min<int64_t>(*nterms, (int64_t)t.size());
      for (int64_t i = 0; i < n; ++i) terms[i] = tdvp_term{t[i].kind, t[i].out, t[i].in, t[i].env, t[i].coef};
    }
    *nterms = (int64_t)t.size();
    if (flops) *flops = f;
    return TDVP_OK;
  });
}

int tdvp_u1_env_plan(const tdvp_model* model, int32_t site, int32_t direction, const tdvp_bond* bond_in,
                     const tdvp_bond* bond_out, const tdvp_blocks* env_in, const tdvp_blocks* tensor,
                     const tdvp_blocks* env_out, int64_t* nterms, tdvp_env_term* terms, double* flops) {
  return guarded(nullptr, [&]() -> int {
    EnvInputs in;
    std::string err;
    int rc = u1_load_env_inputs(in, model, site, direction, bond_in, bond_out, env_in, tensor, env_out, err);
    if (rc) return set_error(nullptr, rc, err);
    if (!nterms) return set_error(nullptr, TDVP_E_INVALID, "nterms is null");
    std::vector<ETerm> t;
    double f = 0;
    u1_plan_env(*model, site, direction, in.bin, in.bout, in.ein, in.ten, in.eout, t, f);
    if (terms) {
      const int64_t n = std::min<int64_t>(*nterms, (int64_t)t.size());
      for (int64_t i = 0; i < n; ++i)
        terms[i] = tdvp_env_term{t[i].kind, t[i].out, t[i].bra, t[i].ket, t[i].env, t[i].coef};
    }
    *nterms = (int64_t)t.size();
    if (flops) *flops = f;
    return TDVP_OK;
  });
}

int tdvp_u1_heff_apply(tdvp_ctx* ctx, const tdvp_model* model, int32_t site, int32_t nsites, const tdvp_bond* left,
                       const tdvp_bond* right, const tdvp_blocks* Lenv, const tdvp_blocks* Renv, const tdvp_blocks* x,
                       tdvp_blocks* y) {
  if (!ctx) return set_error(nullptr, TDVP_E_INVALID, "null ctx");
  return guarded(ctx, [&]() -> int {
    HeffInputs in;
    std::string err;
    int rc = u1_load_heff_inputs(in, model, site, nsites, left, right, Lenv, Renv, x, err);
    Blocks yb;
    if (!rc) rc = match_keys(in.x, yb, y, err);
    if (rc) return set_error(ctx, rc, err);
    if ((in.x.n() && (!in.x.data || !yb.data)) || (in.Le.n() && !in.Le.data) || (in.Re.n() && !in.Re.data))
      return set_error(ctx, TDVP_E_INVALID, "null device data pointer");
    TDVP_HIP(ctx, hipSetDevice(ctx->device));
    auto p = heff_program(ctx, *model, site, nsites, in, yb, rc);
    if (rc) return rc;
    Bufs b{};
    b.p[0] = (const double*)in.x.data;
    b.p[1] = (const double*)in.Le.data;
    b.p[2] = (const double*)in.Re.data;
    return launch_gemm(ctx, *p, b, (double*)yb.data, ctx->precision);
  });
}

int tdvp_u1_env_update(tdvp_ctx* ctx, const tdvp_model* model, int32_t site, int32_t direction,
                       const tdvp_bond* bond_in, const tdvp_bond* bond_out, const tdvp_blocks* env_in,
                       const tdvp_blocks* tensor, tdvp_blocks* env_out) {
  if (!ctx) return set_error(nullptr, TDVP_E_INVALID, "null ctx");
  return guarded(ctx, [&]() -> int {
    EnvInputs in;
    std::string err;
    int rc = u1_load_env_inputs(in, model, site, direction, bond_in, bond_out, env_in, tensor, env_out, err);
    if (rc) return set_error(ctx, rc, err);
    if ((in.ten.n() && !in.ten.data) || (in.eout.n() && !in.eout.data) || (in.ein.n() && !in.ein.data))
      return set_error(ctx, TDVP_E_INVALID, "null device data pointer");
    TDVP_HIP(ctx, hipSetDevice(ctx->device));
    return env_update_dev(ctx, *model, site, direction, in);
  });
}

int tdvp_u1_krylov_expm(tdvp_ctx* ctx, const tdvp_model* model, int32_t site, int32_t nsites, const tdvp_bond* left,
                        const tdvp_bond* right, const tdvp_blocks* Lenv, const tdvp_blocks* Renv, tdvp_blocks* x,
                        double tau_re, double tau_im, double tol, int32_t maxdim, tdvp_krylov_info* info) {
  if (!ctx) return set_error(nullptr, TDVP_E_INVALID, "null ctx");
  return guarded(ctx, [&]() -> int {
    HeffInputs in;
    std::string err;
    int rc = u1_load_heff_inputs(in, model, site, nsites, left, right, Lenv, Renv, x, err);
    if (rc) return set_error(ctx, rc, err);
    if (maxdim < 1 || maxdim > 64) return set_error(ctx, TDVP_E_INVALID, "maxdim must be in 1..64");
    if (!(tol >= 0.0)) return set_error(ctx, TDVP_E_INVALID, "tol must be >= 0");
    TDVP_HIP(ctx, hipSetDevice(ctx->device));
    KrylovResult kr;
    rc = krylov_dev(ctx, *model, site, nsites, in, {tau_re, tau_im}, tol, maxdim, kr);
    if (rc == TDVP_OK || rc == TDVP_E_NOCONV || rc == TDVP_E_NONFINITE) {
      bool bad = false;
      if (int r2 = take_bad_flag(ctx, bad)) return r2;
      if (bad && rc != TDVP_E_NONFINITE) rc = set_error(ctx, TDVP_E_NONFINITE, "non-finite values in the Krylov exponential");
    }
    if (info) {
      std::memset(info, 0, sizeof(*info));
      info->iters = kr.iters;
      info->graph_iters = kr.graph_iters;
      info->converged = kr.converged;
      info->err_est = kr.err;
      info->norm_in = kr.norm;
      for (int i = 0; i < kr.iters && i < 64; ++i) info->alpha[i] = kr.alpha[i];
      for (int i = 0; i < kr.iters && i < 64 && i < (int)kr.beta.size(); ++i) info->beta[i] = kr.beta[i];
    }
    return rc;
  });
}

}  // extern "C"

// Host-only entry points of the C ABI: layouts and plans.  No device work.
#include <cstring>
#include <string>

#include "../../include/tdvp.h"
#include "common.hpp"
#include "plan.hpp"

using namespace tdvp;

extern "C" {

int tdvp_center_layout(const tdvp_bond* left, const tdvp_bond* right, int32_t nsites, int32_t* nblocks,
                       int32_t* keys, int64_t* offsets, int64_t* total) {
  return guarded(nullptr, [&]() -> int {
    std::string err;
    if (nsites != 1 && nsites != 2) return set_error(nullptr, TDVP_E_INVALID, "nsites must be 1 or 2");
    if (!nblocks) return set_error(nullptr, TDVP_E_INVALID, "nblocks is null");
    Bond l, r;
    int rc = load_bond(l, left, err);
    if (!rc) rc = load_bond(r, right, err);
    if (rc) return set_error(nullptr, rc, err);
    Blocks b;
    layout_center(l, r, nsites, b);
    *nblocks = b.n();
    if (total) *total = b.size;
    if (keys) std::memcpy(keys, b.key.data(), sizeof(int) * b.key.size());
    if (offsets) std::memcpy(offsets, b.off.data(), sizeof(int64_t) * b.off.size());
    return TDVP_OK;
  });
}

int tdvp_env_layout(const tdvp_bond* bond, int32_t* nblocks, int32_t* keys, int64_t* offsets,
                    int64_t* total) {
  return guarded(nullptr, [&]() -> int {
    std::string err;
    if (!nblocks) return set_error(nullptr, TDVP_E_INVALID, "nblocks is null");
    Bond b;
    int rc = load_bond(b, bond, err);
    if (rc) return set_error(nullptr, rc, err);
    Blocks e;
    layout_env(b, e);
    *nblocks = e.n();
    if (total) *total = e.size;
    if (keys) std::memcpy(keys, e.key.data(), sizeof(int) * e.key.size());
    if (offsets) std::memcpy(offsets, e.off.data(), sizeof(int64_t) * e.off.size());
    return TDVP_OK;
  });
}

int tdvp_heff_plan(const tdvp_model* model, int32_t site, int32_t nsites, const tdvp_bond* left,
                   const tdvp_bond* right, const tdvp_blocks* Lenv, const tdvp_blocks* Renv,
                   const tdvp_blocks* x, int64_t* nterms, tdvp_term* terms, double* flops) {
  return guarded(nullptr, [&]() -> int {
    HeffInputs in;
    std::string err;
    int rc = load_heff_inputs(in, model, site, nsites, left, right, Lenv, Renv, x, err);
    if (rc) return set_error(nullptr, rc, err);
    std::vector<HTerm> t;
    double f = 0;
    plan_heff(*model, site, nsites, in.l, in.r, in.Le, in.Re, in.x, t, f);
    if (!nterms) return set_error(nullptr, TDVP_E_INVALID, "nterms is null");
    int64_t cap = *nterms;
    *nterms = (int64_t)t.size();
    if (flops) *flops = f;
    if (terms)
      for (int64_t i = 0; i < (int64_t)t.size() && i < cap; ++i)
        terms[i] = tdvp_term{t[i].kind, t[i].out, t[i].in, t[i].env, t[i].coef};
    return TDVP_OK;
  });
}

int tdvp_env_plan(const tdvp_model* model, int32_t site, int32_t direction, const tdvp_bond* bond_in,
                  const tdvp_bond* bond_out, const tdvp_blocks* env_in, const tdvp_blocks* tensor,
                  const tdvp_blocks* env_out, int64_t* nterms, tdvp_env_term* terms, double* flops) {
  return guarded(nullptr, [&]() -> int {
    EnvInputs in;
    std::string err;
    int rc = load_env_inputs(in, model, site, direction, bond_in, bond_out, env_in, tensor, env_out, err);
    if (rc) return set_error(nullptr, rc, err);
    std::vector<ETerm> t;
    double f = 0;
    plan_env(*model, site, direction, in.bin, in.bout, in.ein, in.ten, in.eout, t, f);
    if (!nterms) return set_error(nullptr, TDVP_E_INVALID, "nterms is null");
    int64_t cap = *nterms;
    *nterms = (int64_t)t.size();
    if (flops) *flops = f;
    if (terms)
      for (int64_t i = 0; i < (int64_t)t.size() && i < cap; ++i)
        terms[i] = tdvp_env_term{t[i].kind, t[i].out, t[i].bra, t[i].ket, t[i].env, t[i].coef};
    return TDVP_OK;
  });
}

}  // extern "C"

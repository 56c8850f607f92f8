// Error state and argument loading for the C ABI.
#include "common.hpp"

#include "ctx.hpp"

namespace tdvp {

namespace {
thread_local std::string g_err;
}

int set_error(const tdvp_ctx* ctx, int code, const std::string& msg) {
  g_err = msg;
  if (ctx) const_cast<tdvp_ctx*>(ctx)->err = msg;
  return code;
}

const char* get_error(const tdvp_ctx* ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

int load_heff_inputs(HeffInputs& in, const tdvp_model* model, int site, int nsites, const tdvp_bond* left,
                     const tdvp_bond* right, const tdvp_blocks* Lenv, const tdvp_blocks* Renv,
                     const tdvp_blocks* x, std::string& err) {
  if (!model) { err = "null model"; return TDVP_E_INVALID; }
  if (nsites != 1 && nsites != 2) { err = "nsites must be 1 or 2"; return TDVP_E_INVALID; }
  if (model->L < 2 || site < 1 || site + nsites - 1 > model->L) { err = "site out of range"; return TDVP_E_INVALID; }
  int rc = load_bond(in.l, left, err);
  if (!rc) rc = load_bond(in.r, right, err);
  if (!rc) rc = load_env(in.Le, Lenv, in.l, err);
  if (!rc) rc = load_env(in.Re, Renv, in.r, err);
  if (!rc) rc = load_center(in.x, x, in.l, in.r, nsites, err);
  return rc;
}

int load_env_inputs(EnvInputs& in, const tdvp_model* model, int site, int dir, const tdvp_bond* bond_in,
                    const tdvp_bond* bond_out, const tdvp_blocks* env_in, const tdvp_blocks* tensor,
                    const tdvp_blocks* env_out, std::string& err) {
  if (!model) { err = "null model"; return TDVP_E_INVALID; }
  if (dir != 1 && dir != -1) { err = "direction must be +1 or -1"; return TDVP_E_INVALID; }
  if (site < 1 || site > model->L) { err = "site out of range"; return TDVP_E_INVALID; }
  int rc = load_bond(in.bin, bond_in, err);
  if (!rc) rc = load_bond(in.bout, bond_out, err);
  if (!rc) rc = load_env(in.ein, env_in, in.bin, err);
  if (!rc) rc = dir > 0 ? load_site(in.ten, tensor, in.bin, in.bout, err)
                        : load_site(in.ten, tensor, in.bout, in.bin, err);
  if (!rc) rc = load_env(in.eout, env_out, in.bout, err);
  return rc;
}

}  // namespace tdvp

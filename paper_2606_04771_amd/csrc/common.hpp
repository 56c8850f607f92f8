// Error handling and argument loading shared by the C-ABI entry points.
#pragma once

#include <exception>
#include <string>

#include "../../include/tdvp.h"
#include "plan.hpp"

struct tdvp_ctx;

namespace tdvp {

// Records msg as the last error of ctx (or of the calling thread) and
// returns code.
int set_error(const tdvp_ctx* ctx, int code, const std::string& msg);
const char* get_error(const tdvp_ctx* ctx);

// Runs f, turning any C++ exception into an error code (none crosses the ABI).
template <class F>
int guarded(const tdvp_ctx* ctx, F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return set_error(ctx, TDVP_E_NOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return set_error(ctx, TDVP_E_INVALID, std::string("internal error: ") + e.what());
  } catch (...) {
    return set_error(ctx, TDVP_E_INVALID, "internal error");
  }
}

// sym: 0 = U(1) x SU(2) reduced tensors, 1 = the abelian U(1) x U(1) variant
struct HeffInputs {
  Bond l, r;
  Blocks Le, Re, x;
  int sym = 0;
};
int load_heff_inputs(HeffInputs& in, const tdvp_model* model, int site, int nsites, const tdvp_bond* left,
                     const tdvp_bond* right, const tdvp_blocks* Lenv, const tdvp_blocks* Renv,
                     const tdvp_blocks* x, std::string& err);

struct EnvInputs {
  Bond bin, bout;
  Blocks ein, ten, eout;
  int sym = 0;
};
int load_env_inputs(EnvInputs& in, const tdvp_model* model, int site, int dir, const tdvp_bond* bond_in,
                    const tdvp_bond* bond_out, const tdvp_blocks* env_in, const tdvp_blocks* tensor,
                    const tdvp_blocks* env_out, std::string& err);

// The abelian U(1) x U(1) variant (bond q = 2 S^z, tj = N of the left block).
int u1_load_heff_inputs(HeffInputs& in, const tdvp_model* model, int site, int nsites, const tdvp_bond* left,
                        const tdvp_bond* right, const tdvp_blocks* Lenv, const tdvp_blocks* Renv,
                        const tdvp_blocks* x, std::string& err);
int u1_load_env_inputs(EnvInputs& in, const tdvp_model* model, int site, int dir, const tdvp_bond* bond_in,
                       const tdvp_bond* bond_out, const tdvp_blocks* env_in, const tdvp_blocks* tensor,
                       const tdvp_blocks* env_out, std::string& err);

}  // namespace tdvp

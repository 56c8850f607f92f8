// Limits of the in-house Householder tridiagonal reduction (eig.hip) beyond
// the ones declared with its entry points.
#pragma once

#include <cstdint>

struct tdvp_ctx;

namespace tdvp {

// Matrices of n in (1024, kTrdMaxNLarge] run with six rows of [k, n) per
// thread and 3 n complex values of LDS per workgroup (~76 KB at 1536).
constexpr int64_t kTrdMaxNLarge = 1536;

// Largest n the reduction takes on the context's device: kTrdMaxNLarge when
// a workgroup may hold that much LDS, else 1024.
int64_t eig_trd_max_n(tdvp_ctx* ctx);

}  // namespace tdvp

// Symmetry algebra of the U(1)_spin x SU(2)_charge reduced Hubbard chain.
//
// The paper groups pseudospin multiplets into reduced elements by the
// Wigner-Eckart theorem (supplementary section S2.1).  Every recoupling
// coefficient the hot path needs is computed here numerically, in FP64, by
// contracting Clebsch-Gordan coupling tensors with the local operators
// written in the multiplet basis; nothing depends on a closed-form 6j table.
#pragma once

#include <array>
#include <cstdint>
#include <unordered_map>
#include <vector>

namespace tdvp {

// Clebsch-Gordan <j1 m1; j2 m2 | J M>, Condon-Shortley phase, all arguments
// doubled (tj = 2j, tm = 2m).  Racah's formula in long double.
double clebsch(int tj1, int tm1, int tj2, int tm2, int tJ, int tM);

// Local multiplets s = 0,1,2 of a Hubbard site: (q, tj) and first component
// in the 4-component multiplet basis (s0 m=+1/2, s0 m=-1/2, s1, s2).
constexpr int kLocQ[3] = {0, 1, -1};
constexpr int kLocTJ[3] = {1, 0, 0};
constexpr int kLocC0[3] = {0, 2, 3};
// Environment channels w = 0 'H', 1 'D+', 2 'D-': (q_w, tj_w).
constexpr int kChQ[3] = {0, 1, -1};
constexpr int kChTJ[3] = {0, 1, 1};

inline bool triangle(int ta, int tb, int tc) {
  return tc >= (ta > tb ? ta - tb : tb - ta) && tc <= ta + tb && ((ta + tb + tc) & 1) == 0;
}

using Mat4 = std::array<double, 16>;    // row-major 4x4 in the multiplet basis
using Mat16 = std::array<double, 256>;  // row-major 16x16, site 1 slow

// Operators of site k (1-based) in the multiplet basis.
struct SiteOps {
  Mat4 left[3][2];   // left-edge doublet components O^w_kappa (w = 1, 2; kappa = +1/2, -1/2)
  Mat4 right[3][2];  // partner components Q^w_kappa
  Mat4 onsite;       // U (n_up - 1/2)(n_dn - 1/2)
};
SiteOps site_ops(int k, double U);
// -t sum_s (c+_{k s} c_{k+1 s} + h.c.) in the multiplet basis of sites k, k+1.
Mat16 bond_hop(int k, double t);

// Recoupling coefficients (see symm.cpp for the contraction each one is).
// Labels: tj of bond sectors, s of local multiplets, w of channels.
struct Coeffs {
  double t, U;
  // two-site block (a, s1, x, s2, b)
  double left_hop(int site, int w, int tja_out, int s1_out, int tja_in, int s1_in, int tjx, int s2,
                  int tjb);
  double right_hop(int site, int w, int tja, int s1, int tjx, int s2_out, int tjb_out, int s2_in,
                   int tjb_in);
  double mid_hop(int site, int tja, int s1o, int tjxo, int s2o, int s1i, int tjxi, int s2i, int tjb);
  double onsite2(int s1, int s2) const;
  // one-site block (a, s, b) at site k
  double left_hop1(int site, int w, int tja_out, int s_out, int tja_in, int s_in, int tjb);
  double right_hop1(int site, int w, int tja, int s_out, int tjb_out, int s_in, int tjb_in);
  double onsite1(int s) const;
  // environment updates.  Left: new env block (b', w', b) from A(a',s',b')^dag
  // [E(a', w, a)] A(a, s, b); w = -1 for the identity channel.
  double env_left(int site, int w_out, int tjb_out, int tjb_in, int w_in, int tja_out, int s_out,
                  int tja_in, int s_in);
  // Right: new env block (x', w', x) from conj B(x',s',b') [E(b', w, b)] B(x, s, b)^T.
  double env_right(int site, int w_out, int tjx_out, int tjx_in, int w_in, int tjb_out, int s_out,
                   int tjb_in, int s_in);

  std::unordered_map<uint64_t, double> cache;
};

}  // namespace tdvp

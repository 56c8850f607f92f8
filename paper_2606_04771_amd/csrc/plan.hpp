// Host-side bookkeeping of the reduced block-sparse tensors: bonds, block
// lists, validation against the fusion rules, canonical layouts, and the term
// lists of the effective-Hamiltonian apply and of the environment updates.
#pragma once

#include <cstdint>
#include <map>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/tdvp.h"
#include "symm.hpp"

namespace tdvp {

struct Bond {
  std::vector<int> q, tj;
  std::vector<int64_t> d;
  std::map<std::pair<int, int>, int> index;
  int size() const { return (int)q.size(); }
  int find(int qq, int tt) const {
    auto it = index.find({qq, tt});
    return it == index.end() ? -1 : it->second;
  }
  void add(int qq, int tt, int64_t dd) {
    index[{qq, tt}] = (int)q.size();
    q.push_back(qq);
    tj.push_back(tt);
    d.push_back(dd);
  }
  int64_t chi_full() const {
    int64_t s = 0;
    for (int i = 0; i < size(); ++i) s += d[i] * (tj[i] + 1);
    return s;
  }
  int64_t chi_su2() const {
    int64_t s = 0;
    for (auto v : d) s += v;
    return s;
  }
};

int load_bond(Bond& b, const tdvp_bond* in, std::string& err);

// Block list: key of keylen ints per block, element offset, dims.
struct Blocks {
  int keylen = 0;
  std::vector<int> key;
  std::vector<int64_t> off, rows, cols;
  std::unordered_map<uint64_t, int> map;
  int64_t size = 0;
  void* data = nullptr;
  int n() const { return (int)off.size(); }
  const int* k(int i) const { return &key[(size_t)i * keylen]; }
  int find(const int* kk) const;
  int find3(int a, int b, int c) const { int kk[3] = {a, b, c}; return find(kk); }
  int find5(int a, int b, int c, int d, int e) const { int kk[5] = {a, b, c, d, e}; return find(kk); }
  void push(const int* kk, int64_t o, int64_t r, int64_t c);
};

// Centre tensor between bonds l and r (nsites 1: (ia, s, ib); 2: (ia, s1, tjx, s2, ib)).
int load_center(Blocks& B, const tdvp_blocks* in, const Bond& l, const Bond& r, int nsites,
                std::string& err);
// One-site tensor (A or B) between bonds l and r.
int load_site(Blocks& B, const tdvp_blocks* in, const Bond& l, const Bond& r, std::string& err);
// Environment on bond b: (iout, w, iin).
int load_env(Blocks& B, const tdvp_blocks* in, const Bond& b, std::string& err);
// Check that y lists the same keys as x (offsets may differ).
int match_keys(const Blocks& x, Blocks& y, const tdvp_blocks* in, std::string& err);

void layout_center(const Bond& l, const Bond& r, int nsites, Blocks& out);
void layout_env(const Bond& b, Blocks& out);
void layout_site(const Bond& l, const Bond& r, Blocks& out);

struct HTerm {
  int kind, out, in, env;
  double coef;
};
struct ETerm {
  int kind, out, bra, ket, env;
  double coef;
};

Coeffs& coeffs_for(double t, double U);

// Effective Hamiltonian of sites site..site+nsites-1 on x (terms index x's
// blocks for both in and out, and Le/Re blocks for env).
void plan_heff(const tdvp_model& m, int site, int nsites, const Bond& l, const Bond& r,
               const Blocks& Le, const Blocks& Re, const Blocks& x, std::vector<HTerm>& terms,
               double& flops);
// Environment update (direction +1 left, -1 right).
void plan_env(const tdvp_model& m, int site, int dir, const Bond& bin, const Bond& bout,
              const Blocks& ein, const Blocks& ten, const Blocks& eout, std::vector<ETerm>& terms,
              double& flops);

// The abelian U(1) x U(1) variant (abelian.cpp): bond sectors (q = 2 S^z,
// tj = N), local states s = 0..3, keys (ia, s, ib) and (ia, s1, s2, ib),
// environment channels w = 0..4.
int u1_load_bond(Bond& b, const tdvp_bond* in, std::string& err);
int u1_load_center(Blocks& B, const tdvp_blocks* in, const Bond& l, const Bond& r, int nsites, std::string& err);
int u1_load_env(Blocks& B, const tdvp_blocks* in, const Bond& b, std::string& err);
void u1_layout_center(const Bond& l, const Bond& r, int nsites, Blocks& out);
void u1_layout_env(const Bond& b, Blocks& out);
void u1_plan_heff(const tdvp_model& m, int site, int nsites, const Bond& l, const Bond& r, const Blocks& Le,
                  const Blocks& Re, const Blocks& x, std::vector<HTerm>& terms, double& flops);
void u1_plan_env(const tdvp_model& m, int site, int dir, const Bond& bin, const Bond& bout, const Blocks& ein,
                 const Blocks& ten, const Blocks& eout, std::vector<ETerm>& terms, double& flops);

}  // namespace tdvp

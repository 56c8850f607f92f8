// U(1)_N x U(1)_Sz symmetric Hubbard chain: the abelian special case of the
// reduced hot path (the paper's U(1)xU(1) comparison, Table 1 and Table S1).
//
// Bond sectors are (N, 2S^z) of everything left of the bond, each of
// dimension one in the local space, so there is no recoupling: every
// coefficient is a matrix element of a local operator in the occupation
// basis s = n_up + 2 n_dn (0 = |0>, 1 = |up>, 2 = |dn>, 3 = |up dn> =
// c+_up c+_dn |0>, Jordan-Wigner mode order 1up, 1dn, 2up, ...).  The
// environments carry the block Hamiltonian (channel 0) and, one channel per
// component, the edge operators of the pseudospin doublets the SU(2) path
// uses: channel 1, 2 = D+ components (c+_up P, (-1)^k c_dn P), channel 3, 4 =
// D- components (c+_dn P, -(-1)^k c_up P) on the last site k of a left block,
// and their partners on the first site of a right block.  These are the six
// channels (identity implicit) of the abelian MPO.  The block products are
// the same grouped GEMM programs as the SU(2) path's.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "common.hpp"
#include "plan.hpp"

namespace tdvp {

namespace {

constexpr int kN[4] = {0, 1, 1, 2};
constexpr int kSz[4] = {0, 1, -1, 0};
// (N, 2S^z) carried by channel w (the edge operator); 0 is the Hamiltonian
constexpr int kWN[5] = {0, 1, -1, 1, -1};
constexpr int kWSz[5] = {0, 1, 1, -1, -1};
// D+ channels enter the bond hopping with +, D- channels with -
constexpr double kWSign[5] = {0.0, 1.0, 1.0, -1.0, -1.0};

typedef double M4[4][4];

// annihilators in the occupation basis; the down one carries the on-site
// string (-1)^{n_up}
void a_up(M4 m) {
  std::memset(m, 0, sizeof(M4));
  m[0][1] = 1.0;
  m[2][3] = 1.0;
}
void a_dn(M4 m) {
  std::memset(m, 0, sizeof(M4));
  m[0][2] = 1.0;
  m[1][3] = -1.0;
}
const double kParity[4] = {1.0, -1.0, -1.0, 1.0};

// Left-edge operator of channel w on site k: m[out][in].
void left_op(int w, int k, M4 m) {
  M4 a;
  const double sg = (k % 2 == 0) ? 1.0 : -1.0;
  double f = 1.0;
  bool dag = false;
  switch (w) {
    case 1: a_up(a); dag = true; break;            // c+_up P
    case 2: a_dn(a); f = sg; break;                 // (-1)^k c_dn P
    case 3: a_dn(a); dag = true; break;            // c+_dn P
    default: a_up(a); f = -sg; break;               // -(-1)^k c_up P
  }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) m[i][j] = f * (dag ? a[j][i] : a[i][j]) * kParity[j];
}

// Partner of channel w on site k, the first site of a right block:
// eps(kappa) times the opposite doublet's -kappa component, without parity.
void right_op(int w, int k, M4 m) {
  M4 a;
  const double sg = (k % 2 == 0) ? 1.0 : -1.0;
  double f = 1.0;
  bool dag = false;
  switch (w) {
    case 1: a_up(a); f = -sg; break;                // -(-1)^k c_up
    case 2: a_dn(a); f = -1.0; dag = true; break;   // -c+_dn
    case 3: a_dn(a); f = sg; break;                 // (-1)^k c_dn
    default: a_up(a); f = -1.0; dag = true; break;  // -c+_up
  }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) m[i][j] = f * (dag ? a[j][i] : a[i][j]);
}

double onsite(int s, double U) {   // U (n_up - 1/2)(n_dn - 1/2), diagonal
  const double nu = (s & 1) ? 0.5 : -0.5, nd = (s & 2) ? 0.5 : -0.5;
  return U * nu * nd;
}

// -t sum_sigma (c+_{1 sigma} c_{2 sigma} + h.c.) on two sites, as
// h[(s1', s2')][(s1, s2)], from the mode-ordered Jordan-Wigner action on the
// occupation bits (modes 1up, 1dn, 2up, 2dn = bits 0..3).
void two_site_hop(double t, double h[16][16]) {
  std::memset(h, 0, sizeof(double) * 256);
  auto apply = [](int occ, int mode, bool create, int& out, double& sign) -> bool {
    const bool filled = (occ >> mode) & 1;
    if (filled == create) return false;
    int before = 0;
    for (int b = 0; b < mode; ++b) before += (occ >> b) & 1;
    sign *= (before & 1) ? -1.0 : 1.0;
    out = occ ^ (1 << mode);
    return true;
  };
  for (int s1 = 0; s1 < 4; ++s1)
    for (int s2 = 0; s2 < 4; ++s2) {
      const int occ = s1 | (s2 << 2);
      for (int sp = 0; sp < 2; ++sp)
        for (int dir = 0; dir < 2; ++dir) {   // c+_1 c_2 and c+_2 c_1
          const int mc = dir == 0 ? sp : 2 + sp, ma = dir == 0 ? 2 + sp : sp;
          int o1, o2;
          double sign = 1.0;
          if (!apply(occ, ma, false, o1, sign)) continue;
          if (!apply(o1, mc, true, o2, sign)) continue;
          h[(o2 & 3) * 4 + (o2 >> 2)][s1 * 4 + s2] += -t * sign;
        }
    }
}

int fail(std::string& err, int code, const std::string& msg) {
  err = msg;
  return code;
}

int load_blocks(Blocks& B, const tdvp_blocks* in, int keylen, std::string& err) {
  if (!in) return fail(err, TDVP_E_INVALID, "null block descriptor");
  if (in->nblocks < 0 || (in->nblocks > 0 && (!in->keys || !in->offsets)))
    return fail(err, TDVP_E_INVALID, "block descriptor arrays missing");
  B = Blocks();
  B.keylen = keylen;
  B.size = in->size;
  B.data = in->data;
  return TDVP_OK;
}

int check_offsets(Blocks& B, std::string& err) {
  std::vector<std::pair<int64_t, int64_t>> iv;
  for (int i = 0; i < B.n(); ++i) {
    const int64_t len = B.rows[i] * B.cols[i];
    if (B.off[i] < 0 || B.off[i] + len > B.size) return fail(err, TDVP_E_SHAPE, "block outside data");
    iv.push_back({B.off[i], B.off[i] + len});
  }
  std::sort(iv.begin(), iv.end());
  for (size_t i = 1; i < iv.size(); ++i)
    if (iv[i].first < iv[i - 1].second) return fail(err, TDVP_E_SHAPE, "overlapping blocks");
  return TDVP_OK;
}

}  // namespace

int u1_load_bond(Bond& b, const tdvp_bond* in, std::string& err) {
  if (!in) return fail(err, TDVP_E_INVALID, "null bond");
  if (in->n < 0 || (in->n > 0 && (!in->q || !in->tj || !in->dim)))
    return fail(err, TDVP_E_INVALID, "bond arrays missing");
  b = Bond();
  for (int i = 0; i < in->n; ++i) {
    if (in->tj[i] < 0 || in->dim[i] <= 0 || std::abs(in->q[i]) > in->tj[i] || in->tj[i] > 100000 ||
        ((in->tj[i] - in->q[i]) & 1))
      return fail(err, TDVP_E_SECTOR, "bad (N, 2Sz) bond sector");
    if (b.find(in->q[i], in->tj[i]) >= 0) return fail(err, TDVP_E_SECTOR, "repeated bond sector");
    b.add(in->q[i], in->tj[i], in->dim[i]);
  }
  return TDVP_OK;
}

int u1_load_center(Blocks& B, const tdvp_blocks* in, const Bond& l, const Bond& r, int nsites, std::string& err) {
  const int kl = nsites == 2 ? 4 : 3;
  int rc = load_blocks(B, in, kl, err);
  if (rc) return rc;
  for (int i = 0; i < in->nblocks; ++i) {
    const int* k = in->keys + (size_t)i * kl;
    const int ia = k[0], ib = k[kl - 1];
    if (ia < 0 || ia >= l.size() || ib < 0 || ib >= r.size())
      return fail(err, TDVP_E_SECTOR, "block key refers to a missing sector");
    for (int j = 1; j < kl - 1; ++j)
      if (k[j] < 0 || k[j] > 3) return fail(err, TDVP_E_SECTOR, "bad local state");
    const int dn = kN[k[1]] + (nsites == 2 ? kN[k[2]] : 0), ds = kSz[k[1]] + (nsites == 2 ? kSz[k[2]] : 0);
    if (l.tj[ia] + dn != r.tj[ib] || l.q[ia] + ds != r.q[ib])
      return fail(err, TDVP_E_SECTOR, "block violates (N, Sz) conservation");
    if (B.find(k) >= 0) return fail(err, TDVP_E_SECTOR, "repeated block key");
    B.push(k, in->offsets[i], l.d[ia], r.d[ib]);
  }
  return check_offsets(B, err);
}

int u1_load_env(Blocks& B, const tdvp_blocks* in, const Bond& b, std::string& err) {
  int rc = load_blocks(B, in, 3, err);
  if (rc) return rc;
  for (int i = 0; i < in->nblocks; ++i) {
    const int* k = in->keys + (size_t)i * 3;
    const int io = k[0], w = k[1], ii = k[2];
    if (io < 0 || io >= b.size() || ii < 0 || ii >= b.size() || w < 0 || w > 4)
      return fail(err, TDVP_E_SECTOR, "environment key refers to a missing sector or channel");
    if (b.tj[io] != b.tj[ii] + kWN[w] || b.q[io] != b.q[ii] + kWSz[w])
      return fail(err, TDVP_E_SECTOR, "environment block violates the selection rules");
    if (B.find(k) >= 0) return fail(err, TDVP_E_SECTOR, "repeated environment key");
    B.push(k, in->offsets[i], b.d[io], b.d[ii]);
  }
  return check_offsets(B, err);
}

void u1_layout_center(const Bond& l, const Bond& r, int nsites, Blocks& out) {
  out = Blocks();
  out.keylen = nsites == 2 ? 4 : 3;
  int64_t o = 0;
  for (int ia = 0; ia < l.size(); ++ia)
    for (int s1 = 0; s1 < 4; ++s1)
      for (int s2 = 0; s2 < (nsites == 2 ? 4 : 1); ++s2)
        for (int ib = 0; ib < r.size(); ++ib) {
          const int dn = kN[s1] + (nsites == 2 ? kN[s2] : 0), ds = kSz[s1] + (nsites == 2 ? kSz[s2] : 0);
          if (l.tj[ia] + dn != r.tj[ib] || l.q[ia] + ds != r.q[ib]) continue;
          if (nsites == 2) {
            int k[4] = {ia, s1, s2, ib};
            out.push(k, o, l.d[ia], r.d[ib]);
          } else {
            int k[3] = {ia, s1, ib};
            out.push(k, o, l.d[ia], r.d[ib]);
          }
          o += l.d[ia] * r.d[ib];
        }
  out.size = o;
}

void u1_layout_env(const Bond& b, Blocks& out) {
  out = Blocks();
  out.keylen = 3;
  int64_t o = 0;
  for (int w = 0; w < 5; ++w)
    for (int ii = 0; ii < b.size(); ++ii)
      for (int io = 0; io < b.size(); ++io)
        if (b.tj[io] == b.tj[ii] + kWN[w] && b.q[io] == b.q[ii] + kWSz[w]) {
          int k[3] = {io, w, ii};
          out.push(k, o, b.d[io], b.d[ii]);
          o += b.d[io] * b.d[ii];
        }
  out.size = o;
}

// Terms of the effective Hamiltonian of sites site..site+nsites-1 (kinds as
// in plan_heff): the Hamiltonian channels of both environments, the on-site
// interaction and (two sites) the hopping inside the pair as direct terms,
// and the hoppings across the two outer bonds as environment products with
// the partner operators on the sites next to them.
void u1_plan_heff(const tdvp_model& m, int site, int nsites, const Bond& l, const Bond& r, const Blocks& Le,
                  const Blocks& Re, const Blocks& x, std::vector<HTerm>& terms, double& flops) {
  terms.clear();
  flops = 0.0;
  const double t = m.t, U = m.U;
  const int kl = x.keylen;
  const int last = site + nsites - 1;
  M4 q[5], o[5];
  for (int w = 1; w < 5; ++w) {
    right_op(w, site, q[w]);   // partner on the first site, for the bond (site-1, site)
    left_op(w, last, o[w]);    // edge operator on the last site, for the bond (last, last+1)
  }
  const double sgl = (site - 1) % 2 == 0 ? 1.0 : -1.0;   // (-1)^(site-1)
  const double sgr = last % 2 == 0 ? 1.0 : -1.0;         // (-1)^last
  double h2[16][16];
  if (nsites == 2) two_site_hop(t, h2);
  int key[4];
  for (int in = 0; in < x.n(); ++in) {
    const int* k = x.k(in);
    const int a = k[0], b = k[kl - 1], s1 = k[1], s2 = nsites == 2 ? k[2] : 0;
    const double M = (double)x.rows[in], N = (double)x.cols[in];
    // left Hamiltonian channel
    int e = Le.find3(a, 0, a);
    if (e >= 0) {
      terms.push_back({0, in, in, e, 1.0});
      flops += 8.0 * M * M * N;
    }
    e = Re.find3(b, 0, b);
    if (e >= 0) {
      terms.push_back({1, in, in, e, 1.0});
      flops += 8.0 * M * N * N;
    }
    // on-site interaction
    double u = onsite(s1, U) + (nsites == 2 ? onsite(s2, U) : 0.0);
    if (u != 0.0) terms.push_back({2, in, in, -1, u});
    // hopping inside the pair
    if (nsites == 2)
      for (int s1o = 0; s1o < 4; ++s1o)
        for (int s2o = 0; s2o < 4; ++s2o) {
          const double c = h2[s1o * 4 + s2o][s1 * 4 + s2];
          if (c == 0.0) continue;
          key[0] = a; key[1] = s1o; key[2] = s2o; key[3] = b;
          const int out = x.find(key);
          if (out >= 0) terms.push_back({2, out, in, -1, c});
        }
    // hopping across (site-1, site): L_w (a', a) x q_w on the first site
    for (int w = 1; w < 5; ++w)
      for (int so = 0; so < 4; ++so) {
        const double c = q[w][so][s1];
        if (c == 0.0) continue;
        for (int ao = 0; ao < l.size(); ++ao) {
          const int ee = Le.find3(ao, w, a);
          if (ee < 0) continue;
          key[0] = ao; key[1] = so;
          if (nsites == 2) { key[2] = s2; key[3] = b; } else { key[2] = b; }
          const int out = x.find(key);
          if (out < 0) continue;
          terms.push_back({0, out, in, ee, -t * sgl * kWSign[w] * c});
          flops += 8.0 * (double)l.d[ao] * M * N;
        }
      }
    // hopping across (last, last+1): o_w on the last site x R_w (b', b)
    const int sl = nsites == 2 ? s2 : s1;
    for (int w = 1; w < 5; ++w)
      for (int so = 0; so < 4; ++so) {
        const double c = o[w][so][sl];
        if (c == 0.0) continue;
        for (int bo = 0; bo < r.size(); ++bo) {
          const int ee = Re.find3(bo, w, b);
          if (ee < 0) continue;
          key[0] = a;
          if (nsites == 2) { key[1] = s1; key[2] = so; key[3] = bo; } else { key[1] = so; key[2] = bo; }
          const int out = x.find(key);
          if (out < 0) continue;
          terms.push_back({1, out, in, ee, -t * sgr * kWSign[w] * c});
          flops += 8.0 * M * N * (double)r.d[bo];
        }
      }
  }
}

// Terms of one environment update (kinds as in plan_env).  Left (dir +1), new
// block (b', w', b) from A(a', s', b')^dag [.] A(a, s, b): the old Hamiltonian
// channel carried through, the on-site term and the hopping across
// (site-1, site) for w' = 0, and the edge operators of this site for w' > 0.
// Right (dir -1), new block (x', w', x) from conj B(x', s', b') [.] B(x, s, b)^T.
void u1_plan_env(const tdvp_model& m, int site, int dir, const Bond& bin, const Bond& bout, const Blocks& ein,
                 const Blocks& ten, const Blocks& eout, std::vector<ETerm>& terms, double& flops) {
  terms.clear();
  flops = 0.0;
  const double t = m.t, U = m.U;
  M4 hop_op[5], edge_op[5];
  for (int w = 1; w < 5; ++w) {
    if (dir > 0) {
      right_op(w, site, hop_op[w]);   // partners of the old left edge
      left_op(w, site, edge_op[w]);   // new left edge
    } else {
      left_op(w, site, hop_op[w]);    // this site's edge operators meet the old right partners
      right_op(w, site, edge_op[w]);  // new right partners
    }
  }
  const double sg = dir > 0 ? ((site - 1) % 2 == 0 ? 1.0 : -1.0) : (site % 2 == 0 ? 1.0 : -1.0);
  // the tensor's block (a, s, b): for dir +1 a on bin (old), b on bout (new);
  // for dir -1 a on bout (new, x), b on bin (old)
  auto old_of = [&](int blk) { return dir > 0 ? ten.k(blk)[0] : ten.k(blk)[2]; };
  auto new_of = [&](int blk) { return dir > 0 ? ten.k(blk)[2] : ten.k(blk)[0]; };
  const Bond& bo_ = bout;
  for (int bra = 0; bra < ten.n(); ++bra) {
    const int sb = ten.k(bra)[1], ob = old_of(bra), nb = new_of(bra);
    for (int ket = 0; ket < ten.n(); ++ket) {
      const int sk = ten.k(ket)[1], ok = old_of(ket), nk = new_of(ket);
      // the contraction depth: the old bond's sector dimension
      const double dn_b = (double)bo_.d[nb], dn_k = (double)bo_.d[nk];
      // Hamiltonian channel of the new environment: block (nb, 0, nk)
      const int o0 = eout.find3(nb, 0, nk);
      if (o0 >= 0) {
        if (sb == sk) {
          const int e = ein.find3(ob, 0, ok);
          if (e >= 0) {
            terms.push_back({0, o0, bra, ket, e, 1.0});
            flops += 8.0 * ((double)bin.d[ob] * (double)bin.d[ok] * dn_k + (double)bin.d[ob] * dn_b * dn_k);
          }
          if (ob == ok) {
            const double u = onsite(sb, U);
            if (u != 0.0) {
              terms.push_back({1, o0, bra, ket, -1, u});
              flops += 8.0 * (double)bin.d[ob] * dn_b * dn_k;
            }
          }
        }
        for (int w = 1; w < 5; ++w) {
          const double c = hop_op[w][sb][sk];
          if (c == 0.0) continue;
          const int e = ein.find3(ob, w, ok);
          if (e < 0) continue;
          terms.push_back({0, o0, bra, ket, e, -t * sg * kWSign[w] * c});
          flops += 8.0 * ((double)bin.d[ob] * (double)bin.d[ok] * dn_k + (double)bin.d[ob] * dn_b * dn_k);
        }
      }
      // edge channels of the new environment: identity on the old block
      if (ob == ok)
        for (int w = 1; w < 5; ++w) {
          const double c = edge_op[w][sb][sk];
          if (c == 0.0) continue;
          const int ow = eout.find3(nb, w, nk);
          if (ow < 0) continue;
          terms.push_back({1, ow, bra, ket, -1, c});
          flops += 8.0 * (double)bin.d[ob] * dn_b * dn_k;
        }
    }
  }
}

int u1_load_heff_inputs(HeffInputs& in, const tdvp_model* model, int site, int nsites, const tdvp_bond* left,
                        const tdvp_bond* right, const tdvp_blocks* Lenv, const tdvp_blocks* Renv,
                        const tdvp_blocks* x, std::string& err) {
  if (!model) return fail(err, TDVP_E_INVALID, "null model");
  if (nsites != 1 && nsites != 2) return fail(err, TDVP_E_INVALID, "nsites must be 1 or 2");
  if (model->L < 2 || site < 1 || site + nsites - 1 > model->L) return fail(err, TDVP_E_INVALID, "site out of range");
  in.sym = 1;
  int rc = u1_load_bond(in.l, left, err);
  if (!rc) rc = u1_load_bond(in.r, right, err);
  if (!rc) rc = u1_load_env(in.Le, Lenv, in.l, err);
  if (!rc) rc = u1_load_env(in.Re, Renv, in.r, err);
  if (!rc) rc = u1_load_center(in.x, x, in.l, in.r, nsites, err);
  return rc;
}

int u1_load_env_inputs(EnvInputs& in, const tdvp_model* model, int site, int dir, const tdvp_bond* bond_in,
                       const tdvp_bond* bond_out, const tdvp_blocks* env_in, const tdvp_blocks* tensor,
                       const tdvp_blocks* env_out, std::string& err) {
  if (!model) return fail(err, TDVP_E_INVALID, "null model");
  if (dir != 1 && dir != -1) return fail(err, TDVP_E_INVALID, "direction must be +1 or -1");
  if (site < 1 || site > model->L) return fail(err, TDVP_E_INVALID, "site out of range");
  in.sym = 1;
  int rc = u1_load_bond(in.bin, bond_in, err);
  if (!rc) rc = u1_load_bond(in.bout, bond_out, err);
  if (!rc) rc = u1_load_env(in.ein, env_in, in.bin, err);
  if (!rc) rc = dir > 0 ? u1_load_center(in.ten, tensor, in.bin, in.bout, 1, err)
                        : u1_load_center(in.ten, tensor, in.bout, in.bin, 1, err);
  if (!rc) rc = u1_load_env(in.eout, env_out, in.bout, err);
  return rc;
}

}  // namespace tdvp

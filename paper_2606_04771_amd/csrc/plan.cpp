// Block bookkeeping and term lists (see plan.hpp).
#include "plan.hpp"

#include <cmath>
#include <mutex>
#include <set>
#include <sstream>

namespace tdvp {

namespace {

uint64_t hkey(const int* k, int n) {
  uint64_t h = 1469598103934665603ull;
  for (int i = 0; i < n; ++i) {
    h ^= (uint64_t)(uint32_t)(k[i] + 4096);
    h *= 1099511628211ull;
  }
  return h;
}

int fail(std::string& err, int code, const std::string& msg) {
  err = msg;
  return code;
}

}  // namespace

int Blocks::find(const int* kk) const {
  auto it = map.find(hkey(kk, keylen));
  if (it == map.end()) return -1;
  // guard against hash collisions
  const int* s = k(it->second);
  for (int i = 0; i < keylen; ++i)
    if (s[i] != kk[i]) return -1;
  return it->second;
}

void Blocks::push(const int* kk, int64_t o, int64_t r, int64_t c) {
  map[hkey(kk, keylen)] = n();
  key.insert(key.end(), kk, kk + keylen);
  off.push_back(o);
  rows.push_back(r);
  cols.push_back(c);
}

int load_bond(Bond& b, const tdvp_bond* in, std::string& err) {
  if (!in) return fail(err, TDVP_E_INVALID, "null bond");
  if (in->n < 0 || (in->n > 0 && (!in->q || !in->tj || !in->dim)))
    return fail(err, TDVP_E_INVALID, "bond arrays missing");
  b = Bond();
  for (int i = 0; i < in->n; ++i) {
    if (in->tj[i] < 0 || in->dim[i] <= 0 || in->tj[i] > 60 || std::abs(in->q[i]) > 1000)
      return fail(err, TDVP_E_SECTOR, "bad bond sector");
    if (b.find(in->q[i], in->tj[i]) >= 0) return fail(err, TDVP_E_SECTOR, "repeated bond sector");
    b.add(in->q[i], in->tj[i], in->dim[i]);
  }
  return TDVP_OK;
}

static int load_common(Blocks& B, const tdvp_blocks* in, int keylen, std::string& err) {
  if (!in) return fail(err, TDVP_E_INVALID, "null block descriptor");
  if (in->nblocks < 0 || (in->nblocks > 0 && (!in->keys || !in->offsets)))
    return fail(err, TDVP_E_INVALID, "block descriptor arrays missing");
  B = Blocks();
  B.keylen = keylen;
  B.size = in->size;
  B.data = in->data;
  return TDVP_OK;
}

static int finish_blocks(Blocks& B, std::string& err) {
  // offsets in range and non-overlapping
  std::vector<std::pair<int64_t, int64_t>> iv;
  for (int i = 0; i < B.n(); ++i) {
    int64_t len = B.rows[i] * B.cols[i];
    if (B.off[i] < 0 || B.off[i] + len > B.size) return fail(err, TDVP_E_SHAPE, "block outside data");
    iv.push_back({B.off[i], B.off[i] + len});
  }
  std::sort(iv.begin(), iv.end());
  for (size_t i = 1; i < iv.size(); ++i)
    if (iv[i].first < iv[i - 1].second) return fail(err, TDVP_E_SHAPE, "overlapping blocks");
  return TDVP_OK;
}

int load_center(Blocks& B, const tdvp_blocks* in, const Bond& l, const Bond& r, int nsites,
                std::string& err) {
  int kl = nsites == 2 ? 5 : 3;
  int rc = load_common(B, in, kl, err);
  if (rc) return rc;
  for (int i = 0; i < in->nblocks; ++i) {
    const int* k = in->keys + (size_t)i * kl;
    int ia = k[0], ib = k[kl - 1];
    if (ia < 0 || ia >= l.size() || ib < 0 || ib >= r.size())
      return fail(err, TDVP_E_SECTOR, "block key refers to a missing sector");
    if (nsites == 2) {
      int s1 = k[1], tjx = k[2], s2 = k[3];
      if (s1 < 0 || s1 > 2 || s2 < 0 || s2 > 2) return fail(err, TDVP_E_SECTOR, "bad local multiplet");
      if (l.q[ia] + kLocQ[s1] + kLocQ[s2] != r.q[ib] || !triangle(l.tj[ia], kLocTJ[s1], tjx) ||
          !triangle(tjx, kLocTJ[s2], r.tj[ib]))
        return fail(err, TDVP_E_SECTOR, "two-site block violates the fusion rules");
    } else {
      int s = k[1];
      if (s < 0 || s > 2) return fail(err, TDVP_E_SECTOR, "bad local multiplet");
      if (l.q[ia] + kLocQ[s] != r.q[ib] || !triangle(l.tj[ia], kLocTJ[s], r.tj[ib]))
        return fail(err, TDVP_E_SECTOR, "one-site block violates the fusion rules");
    }
    if (B.find(k) >= 0) return fail(err, TDVP_E_SECTOR, "repeated block key");
    B.push(k, in->offsets[i], l.d[ia], r.d[ib]);
  }
  return finish_blocks(B, err);
}

int load_site(Blocks& B, const tdvp_blocks* in, const Bond& l, const Bond& r, std::string& err) {
  return load_center(B, in, l, r, 1, err);
}

int load_env(Blocks& B, const tdvp_blocks* in, const Bond& b, std::string& err) {
  int rc = load_common(B, in, 3, err);
  if (rc) return rc;
  for (int i = 0; i < in->nblocks; ++i) {
    const int* k = in->keys + (size_t)i * 3;
    int io = k[0], w = k[1], ii = k[2];
    if (io < 0 || io >= b.size() || ii < 0 || ii >= b.size() || w < 0 || w > 2)
      return fail(err, TDVP_E_SECTOR, "environment key refers to a missing sector or channel");
    if (b.q[io] != b.q[ii] + kChQ[w] || !triangle(b.tj[ii], kChTJ[w], b.tj[io]))
      return fail(err, TDVP_E_SECTOR, "environment block violates the selection rules");
    if (B.find(k) >= 0) return fail(err, TDVP_E_SECTOR, "repeated environment key");
    B.push(k, in->offsets[i], b.d[io], b.d[ii]);
  }
  return finish_blocks(B, err);
}

int match_keys(const Blocks& x, Blocks& y, const tdvp_blocks* in, std::string& err) {
  int rc = load_common(y, in, x.keylen, err);
  if (rc) return rc;
  if (in->nblocks != x.n()) return fail(err, TDVP_E_SHAPE, "output lists a different number of blocks");
  std::vector<int64_t> off(x.n(), -1);
  for (int i = 0; i < in->nblocks; ++i) {
    int j = x.find(in->keys + (size_t)i * x.keylen);
    if (j < 0 || off[j] >= 0) return fail(err, TDVP_E_SECTOR, "output keys differ from input keys");
    off[j] = in->offsets[i];
  }
  // y indexed like x
  for (int j = 0; j < x.n(); ++j) y.push(x.k(j), off[j], x.rows[j], x.cols[j]);
  return finish_blocks(y, err);
}

void layout_center(const Bond& l, const Bond& r, int nsites, Blocks& out) {
  out = Blocks();
  out.keylen = nsites == 2 ? 5 : 3;
  int64_t o = 0;
  for (int ia = 0; ia < l.size(); ++ia)
    for (int s1 = 0; s1 < 3; ++s1) {
      if (nsites == 1) {
        for (int ib = 0; ib < r.size(); ++ib)
          if (l.q[ia] + kLocQ[s1] == r.q[ib] && triangle(l.tj[ia], kLocTJ[s1], r.tj[ib])) {
            int k[3] = {ia, s1, ib};
            out.push(k, o, l.d[ia], r.d[ib]);
            o += l.d[ia] * r.d[ib];
          }
        continue;
      }
      int t1 = kLocTJ[s1];
      for (int tjx = std::abs(l.tj[ia] - t1); tjx <= l.tj[ia] + t1; tjx += 2)
        for (int s2 = 0; s2 < 3; ++s2)
          for (int ib = 0; ib < r.size(); ++ib)
            if (l.q[ia] + kLocQ[s1] + kLocQ[s2] == r.q[ib] && triangle(tjx, kLocTJ[s2], r.tj[ib])) {
              int k[5] = {ia, s1, tjx, s2, ib};
              out.push(k, o, l.d[ia], r.d[ib]);
              o += l.d[ia] * r.d[ib];
            }
    }
  out.size = o;
}

void layout_site(const Bond& l, const Bond& r, Blocks& out) { layout_center(l, r, 1, out); }

void layout_env(const Bond& b, Blocks& out) {
  out = Blocks();
  out.keylen = 3;
  int64_t o = 0;
  for (int w = 0; w < 3; ++w)
    for (int ii = 0; ii < b.size(); ++ii)
      for (int io = 0; io < b.size(); ++io)
        if (b.q[io] == b.q[ii] + kChQ[w] && triangle(b.tj[ii], kChTJ[w], b.tj[io])) {
          int k[3] = {io, w, ii};
          out.push(k, o, b.d[io], b.d[ii]);
          o += b.d[io] * b.d[ii];
        }
  out.size = o;
}

Coeffs& coeffs_for(double t, double U) {
  static std::mutex mu;
  static std::map<std::pair<double, double>, Coeffs*> all;
  std::lock_guard<std::mutex> g(mu);
  auto& p = all[{t, U}];
  if (!p) {
    p = new Coeffs();
    p->t = t;
    p->U = U;
  }
  return *p;
}

void plan_heff(const tdvp_model& m, int site, int nsites, const Bond& l, const Bond& r,
               const Blocks& Le, const Blocks& Re, const Blocks& x, std::vector<HTerm>& terms,
               double& flops) {
  Coeffs& C = coeffs_for(m.t, m.U);
  terms.clear();
  flops = 0.0;
  const double tiny = 1e-15;
  for (int in = 0; in < x.n(); ++in) {
    const int* k = x.k(in);
    int ia = k[0], ib = k[x.keylen - 1];
    int64_t da = l.d[ia], db = r.d[ib];
    // block Hamiltonians of the two environments (scalar channel, coefficient 1)
    int e = Le.find3(ia, 0, ia);
    if (e >= 0) {
      terms.push_back({0, in, in, e, 1.0});
      flops += 8.0 * da * da * db;
    }
    e = Re.find3(ib, 0, ib);
    if (e >= 0) {
      terms.push_back({1, in, in, e, 1.0});
      flops += 8.0 * da * db * db;
    }
    if (nsites == 2) {
      int s1 = k[1], tjx = k[2], s2 = k[3];
      int qx = l.q[ia] + kLocQ[s1];
      terms.push_back({2, in, in, -1, C.onsite2(s1, s2)});
      // hopping between the two sites: (s1, x, s2) -> (s1', x', s2'), a and b fixed
      for (int s1o = 0; s1o < 3; ++s1o)
        for (int s2o = 0; s2o < 3; ++s2o) {
          if (kLocQ[s1o] + kLocQ[s2o] != kLocQ[s1] + kLocQ[s2]) continue;
          int t1 = kLocTJ[s1o];
          for (int tjxo = std::abs(l.tj[ia] - t1); tjxo <= l.tj[ia] + t1; tjxo += 2) {
            int out = x.find5(ia, s1o, tjxo, s2o, ib);
            if (out < 0) continue;
            double c = C.mid_hop(site, l.tj[ia], s1o, tjxo, s2o, s1, tjx, s2, r.tj[ib]);
            if (std::abs(c) > tiny) terms.push_back({2, out, in, -1, c});
          }
        }
      // hopping across the left bond: L_w(a', a) x partner on site `site`
      for (int w = 1; w <= 2; ++w)
        for (int ao = 0; ao < l.size(); ++ao) {
          int ee = Le.find3(ao, w, ia);
          if (ee < 0) continue;
          for (int s1o = 0; s1o < 3; ++s1o) {
            if (l.q[ao] + kLocQ[s1o] != qx || !triangle(l.tj[ao], kLocTJ[s1o], tjx)) continue;
            int out = x.find5(ao, s1o, tjx, s2, ib);
            if (out < 0) continue;
            double c = C.left_hop(site, w, l.tj[ao], s1o, l.tj[ia], s1, tjx, s2, r.tj[ib]);
            if (std::abs(c) > tiny) {
              terms.push_back({0, out, in, ee, c});
              flops += 8.0 * l.d[ao] * da * db;
            }
          }
        }
      // hopping across the right bond: operator on site+1 x R_w(b', b)
      for (int w = 1; w <= 2; ++w)
        for (int bo = 0; bo < r.size(); ++bo) {
          int ee = Re.find3(bo, w, ib);
          if (ee < 0) continue;
          for (int s2o = 0; s2o < 3; ++s2o) {
            if (qx + kLocQ[s2o] != r.q[bo] || !triangle(tjx, kLocTJ[s2o], r.tj[bo])) continue;
            int out = x.find5(ia, s1, tjx, s2o, bo);
            if (out < 0) continue;
            double c = C.right_hop(site, w, l.tj[ia], s1, tjx, s2o, r.tj[bo], s2, r.tj[ib]);
            if (std::abs(c) > tiny) {
              terms.push_back({1, out, in, ee, c});
              flops += 8.0 * da * db * r.d[bo];
            }
          }
        }
    } else {
      int s = k[1];
      terms.push_back({2, in, in, -1, C.onsite1(s)});
      int qs = l.q[ia] + kLocQ[s];
      (void)qs;
      for (int w = 1; w <= 2; ++w)
        for (int ao = 0; ao < l.size(); ++ao) {
          int ee = Le.find3(ao, w, ia);
          if (ee < 0) continue;
          for (int so = 0; so < 3; ++so) {
            if (l.q[ao] + kLocQ[so] != r.q[ib] || !triangle(l.tj[ao], kLocTJ[so], r.tj[ib])) continue;
            int out = x.find3(ao, so, ib);
            if (out < 0) continue;
            double c = C.left_hop1(site, w, l.tj[ao], so, l.tj[ia], s, r.tj[ib]);
            if (std::abs(c) > tiny) {
              terms.push_back({0, out, in, ee, c});
              flops += 8.0 * l.d[ao] * da * db;
            }
          }
        }
      for (int w = 1; w <= 2; ++w)
        for (int bo = 0; bo < r.size(); ++bo) {
          int ee = Re.find3(bo, w, ib);
          if (ee < 0) continue;
          for (int so = 0; so < 3; ++so) {
            if (l.q[ia] + kLocQ[so] != r.q[bo] || !triangle(l.tj[ia], kLocTJ[so], r.tj[bo])) continue;
            int out = x.find3(ia, so, bo);
            if (out < 0) continue;
            double c = C.right_hop1(site, w, l.tj[ia], so, r.tj[bo], s, r.tj[ib]);
            if (std::abs(c) > tiny) {
              terms.push_back({1, out, in, ee, c});
              flops += 8.0 * da * db * r.d[bo];
            }
          }
        }
    }
  }
}

void plan_env(const tdvp_model& m, int site, int dir, const Bond& bin, const Bond& bout,
              const Blocks& ein, const Blocks& ten, const Blocks& eout, std::vector<ETerm>& terms,
              double& flops) {
  Coeffs& C = coeffs_for(m.t, m.U);
  terms.clear();
  flops = 0.0;
  const double tiny = 1e-15;
  std::set<std::pair<int, int>> stage1;   // (env block, ket block) products
  // tensor blocks grouped by the index on bond_out ("outer" index)
  // dir +1: A keys (ia on bin, s, ib on bout); dir -1: B keys (ix on bout, s, ib on bin)
  std::vector<std::vector<int>> by_outer(bout.size());
  for (int t = 0; t < ten.n(); ++t) {
    const int* k = ten.k(t);
    by_outer[dir > 0 ? k[2] : k[0]].push_back(t);
  }
  for (int o = 0; o < eout.n(); ++o) {
    const int* ok = eout.k(o);
    int po = ok[0], wo = ok[1], pi = ok[2];   // (out sector, channel, in sector) on bond_out
    for (int bra : by_outer[po]) {
      const int* bk = ten.k(bra);
      int inner_b = dir > 0 ? bk[0] : bk[2], sb = bk[1];
      for (int ket : by_outer[pi]) {
        const int* kk = ten.k(ket);
        int inner_k = dir > 0 ? kk[0] : kk[2], sk = kk[1];
        double dout = (double)bout.d[po], din = (double)bout.d[pi];
        if (wo == 0) {
          if (inner_b == inner_k && sb == sk) {
            // carried block Hamiltonian
            int e = ein.find3(inner_k, 0, inner_k);
            if (e >= 0) {
              double c = dir > 0 ? C.env_left(site, 0, bout.tj[po], bout.tj[pi], 0, bin.tj[inner_b], sb,
                                              bin.tj[inner_k], sk)
                                 : C.env_right(site, 0, bout.tj[po], bout.tj[pi], 0, bin.tj[inner_b], sb,
                                               bin.tj[inner_k], sk);
              if (std::abs(c) > tiny) {
                terms.push_back({0, o, bra, ket, e, c});
                double di = (double)bin.d[inner_k];
                if (stage1.insert({e, ket}).second) flops += 8.0 * di * di * din;
                flops += 8.0 * dout * di * din;
              }
            }
            // on-site interaction of the new site
            double c = dir > 0 ? C.env_left(site, 0, bout.tj[po], bout.tj[pi], -1, bin.tj[inner_b], sb,
                                            bin.tj[inner_k], sk)
                               : C.env_right(site, 0, bout.tj[po], bout.tj[pi], -1, bin.tj[inner_b], sb,
                                             bin.tj[inner_k], sk);
            if (std::abs(c) > tiny) {
              terms.push_back({1, o, bra, ket, -1, c});
              flops += 8.0 * dout * (double)bin.d[inner_k] * din;
            }
          }
          // hopping between the old edge and the new site
          for (int w = 1; w <= 2; ++w) {
            int e = ein.find3(inner_b, w, inner_k);
            if (e < 0) continue;
            double c = dir > 0 ? C.env_left(site, 0, bout.tj[po], bout.tj[pi], w, bin.tj[inner_b], sb,
                                            bin.tj[inner_k], sk)
                               : C.env_right(site, 0, bout.tj[po], bout.tj[pi], w, bin.tj[inner_b], sb,
                                             bin.tj[inner_k], sk);
            if (std::abs(c) > tiny) {
              terms.push_back({0, o, bra, ket, e, c});
              double dib = (double)bin.d[inner_b], dik = (double)bin.d[inner_k];
              if (stage1.insert({e, ket}).second) flops += 8.0 * dib * dik * din;
              flops += 8.0 * dout * dib * din;
            }
          }
        } else if (inner_b == inner_k) {
          // new edge operator on the new site
          double c = dir > 0 ? C.env_left(site, wo, bout.tj[po], bout.tj[pi], -1, bin.tj[inner_b], sb,
                                          bin.tj[inner_k], sk)
                             : C.env_right(site, wo, bout.tj[po], bout.tj[pi], -1, bin.tj[inner_b], sb,
                                           bin.tj[inner_k], sk);
          if (std::abs(c) > tiny) {
            terms.push_back({1, o, bra, ket, -1, c});
            flops += 8.0 * dout * (double)bin.d[inner_k] * din;
          }
        }
      }
    }
  }
}

}  // namespace tdvp

// Symmetry algebra: Clebsch-Gordan coefficients, local operators in the
// multiplet basis, and recoupling coefficients by explicit contraction.
#include "symm.hpp"

#include <cmath>
#include <stdexcept>

namespace tdvp {

namespace {

long double lfact(int n2) {  // factorial of a doubled (even) argument
  int n = n2 / 2;
  long double f = 1.0L;
  for (int i = 2; i <= n; ++i) f *= (long double)i;
  return f;
}

}  // namespace

double clebsch(int tj1, int tm1, int tj2, int tm2, int tJ, int tM) {
  if (tm1 + tm2 != tM) return 0.0;
  if (std::abs(tm1) > tj1 || std::abs(tm2) > tj2 || std::abs(tM) > tJ) return 0.0;
  if (((tj1 + tm1) & 1) || ((tj2 + tm2) & 1) || ((tJ + tM) & 1)) return 0.0;
  if (!triangle(tj1, tj2, tJ)) return 0.0;
  // Racah: sqrt((2J+1) D(j1 j2 J) prod of (j +- m)!) * sum_k (-1)^k / (...)
  long double pref = (long double)(tJ + 1) * lfact(tJ + tj1 - tj2) * lfact(tJ - tj1 + tj2) *
                     lfact(tj1 + tj2 - tJ) / lfact(tj1 + tj2 + tJ + 2);
  pref *= lfact(tJ + tM) * lfact(tJ - tM) * lfact(tj1 - tm1) * lfact(tj1 + tm1) *
          lfact(tj2 - tm2) * lfact(tj2 + tm2);
  long double sum = 0.0L;
  for (int k = 0;; ++k) {
    int a0 = tj1 + tj2 - tJ - 2 * k, a1 = tj1 - tm1 - 2 * k, a2 = tj2 + tm2 - 2 * k;
    int a3 = tJ - tj2 + tm1 + 2 * k, a4 = tJ - tj1 - tm2 + 2 * k;
    if (a0 < 0 || a1 < 0 || a2 < 0) break;
    if (a3 < 0 || a4 < 0) continue;
    long double den = lfact(2 * k) * lfact(a0) * lfact(a1) * lfact(a2) * lfact(a3) * lfact(a4);
    sum += ((k & 1) ? -1.0L : 1.0L) / den;
  }
  return (double)(std::sqrt(pref) * sum);
}

// ---------------------------------------------------------------------------
// Local operators.  Jordan-Wigner basis of one site: 0 |0>, 1 |up>, 2 |dn>,
// 3 |up dn> = c+_up c+_dn |0>; a_dn carries the on-site string (-1)^{n_up}.
// Multiplet basis: 0 = (s0, m=+1/2) = |up dn>, 1 = (s0, m=-1/2) = (-1)^k |0>,
// 2 = |up>, 3 = |dn>.
// ---------------------------------------------------------------------------
namespace {

Mat4 zero4() { Mat4 m{}; m.fill(0.0); return m; }
Mat4 mul(const Mat4& a, const Mat4& b) {
  Mat4 c = zero4();
  for (int i = 0; i < 4; ++i)
    for (int k = 0; k < 4; ++k)
      for (int j = 0; j < 4; ++j) c[i * 4 + j] += a[i * 4 + k] * b[k * 4 + j];
  return c;
}
Mat4 tr(const Mat4& a) {
  Mat4 c = zero4();
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) c[j * 4 + i] = a[i * 4 + j];
  return c;
}
Mat4 scale(const Mat4& a, double s) {
  Mat4 c = a;
  for (auto& v : c) v *= s;
  return c;
}

struct JW {
  Mat4 a_up, a_dn, par, n_up, n_dn;
  JW() {
    a_up = zero4();
    a_up[0 * 4 + 1] = 1.0;   // |up> -> |0>
    a_up[2 * 4 + 3] = 1.0;   // |up dn> -> |dn>
    a_dn = zero4();
    a_dn[0 * 4 + 2] = 1.0;   // |dn> -> |0>
    a_dn[1 * 4 + 3] = -1.0;  // c_dn c+_up c+_dn |0> = -|up>
    par = zero4();
    par[0] = 1.0; par[5] = -1.0; par[10] = -1.0; par[15] = 1.0;
    n_up = mul(tr(a_up), a_up);
    n_dn = mul(tr(a_dn), a_dn);
  }
};

// columns: multiplet components, rows: JW states
Mat4 basis(int k) {
  Mat4 u = zero4();
  double p = (k & 1) ? -1.0 : 1.0;
  u[3 * 4 + 0] = 1.0;
  u[0 * 4 + 1] = p;
  u[1 * 4 + 2] = 1.0;
  u[2 * 4 + 3] = 1.0;
  return u;
}

Mat4 to_mult(const Mat4& op, int k) {
  Mat4 u = basis(k);
  return mul(tr(u), mul(op, u));
}

}  // namespace

SiteOps site_ops(int k, double U) {
  JW f;
  SiteOps s{};
  double p = (k & 1) ? -1.0 : 1.0;
  // doublets D+ = (c+_up, p c_dn), D- = (c+_dn, -p c_up) of site k
  Mat4 Dp[2] = {tr(f.a_up), scale(f.a_dn, p)};
  Mat4 Dm[2] = {tr(f.a_dn), scale(f.a_up, -p)};
  for (int kap = 0; kap < 2; ++kap) {
    s.left[1][kap] = to_mult(mul(Dp[kap], f.par), k);
    s.left[2][kap] = to_mult(mul(Dm[kap], f.par), k);
    double eps = kap == 0 ? 1.0 : -1.0;
    s.right[1][kap] = to_mult(scale(Dm[1 - kap], eps), k);
    s.right[2][kap] = to_mult(scale(Dp[1 - kap], eps), k);
  }
  s.left[0][0] = s.left[0][1] = s.right[0][0] = s.right[0][1] = zero4();
  Mat4 e = zero4();
  for (int i = 0; i < 4; ++i) e[i * 5] = 1.0;
  Mat4 a = f.n_up, b = f.n_dn;
  for (int i = 0; i < 16; ++i) { a[i] -= 0.5 * e[i]; b[i] -= 0.5 * e[i]; }
  s.onsite = to_mult(scale(mul(a, b), U), k);
  return s;
}

Mat16 bond_hop(int k, double t) {
  // c+_{k s} c_{k+1 s} = [a+_s P]_k [a_s]_{k+1}, its conjugate [P a_s]_k [a+_s]_{k+1}
  JW f;
  Mat16 h{};
  h.fill(0.0);
  const Mat4* as[2] = {&f.a_up, &f.a_dn};
  for (int sp = 0; sp < 2; ++sp) {
    Mat4 x1 = mul(tr(*as[sp]), f.par), y1 = *as[sp];
    Mat4 x2 = mul(f.par, *as[sp]), y2 = tr(*as[sp]);
    for (int i1 = 0; i1 < 4; ++i1)
      for (int i2 = 0; i2 < 4; ++i2)
        for (int j1 = 0; j1 < 4; ++j1)
          for (int j2 = 0; j2 < 4; ++j2)
            h[(i1 * 4 + i2) * 16 + (j1 * 4 + j2)] +=
                -t * (x1[i1 * 4 + j1] * y1[i2 * 4 + j2] + x2[i1 * 4 + j1] * y2[i2 * 4 + j2]);
  }
  Mat4 u1 = basis(k), u2 = basis(k + 1);
  Mat16 out{};
  out.fill(0.0);
  // out = (u1 x u2)^T h (u1 x u2)
  for (int a1 = 0; a1 < 4; ++a1)
    for (int a2 = 0; a2 < 4; ++a2)
      for (int b1 = 0; b1 < 4; ++b1)
        for (int b2 = 0; b2 < 4; ++b2) {
          double acc = 0.0;
          for (int i1 = 0; i1 < 4; ++i1)
            for (int i2 = 0; i2 < 4; ++i2) {
              double ui = u1[i1 * 4 + a1] * u2[i2 * 4 + a2];
              if (ui == 0.0) continue;
              for (int j1 = 0; j1 < 4; ++j1)
                for (int j2 = 0; j2 < 4; ++j2)
                  acc += ui * h[(i1 * 4 + i2) * 16 + (j1 * 4 + j2)] * u1[j1 * 4 + b1] * u2[j2 * 4 + b2];
            }
          out[(a1 * 4 + a2) * 16 + (b1 * 4 + b2)] = acc;
        }
  return out;
}

// ---------------------------------------------------------------------------
// Coupling tensors.  Magnetic components are indexed in descending order:
// index i <-> tm = tj - 2 i.  Local components use the 4-dim multiplet basis.
// ---------------------------------------------------------------------------
namespace {

inline int tmof(int tj, int i) { return tj - 2 * i; }

// Two-site tree ((a s1)->x) s2 -> b, normalised: T[ma][c1][c2][mb]
struct Tree2 {
  int na, nb;
  std::vector<double> v;
  Tree2(int tja, int s1, int tjx, int s2, int tjb) : na(tja + 1), nb(tjb + 1), v(na * 16 * nb, 0.0) {
    double nrm = 1.0 / std::sqrt((double)(tjb + 1));
    for (int ia = 0; ia < na; ++ia)
      for (int u1 = 0; u1 <= kLocTJ[s1]; ++u1)
        for (int u2 = 0; u2 <= kLocTJ[s2]; ++u2)
          for (int ib = 0; ib < nb; ++ib) {
            int tma = tmof(tja, ia), tm1 = tmof(kLocTJ[s1], u1), tm2 = tmof(kLocTJ[s2], u2);
            int tmx = tma + tm1, tmb = tmof(tjb, ib);
            if (std::abs(tmx) > tjx) continue;
            double c = clebsch(tja, tma, kLocTJ[s1], tm1, tjx, tmx) *
                       clebsch(tjx, tmx, kLocTJ[s2], tm2, tjb, tmb);
            at(ia, kLocC0[s1] + u1, kLocC0[s2] + u2, ib) = c * nrm;
          }
  }
  double& at(int ia, int c1, int c2, int ib) { return v[((ia * 4 + c1) * 4 + c2) * nb + ib]; }
  double at(int ia, int c1, int c2, int ib) const { return v[((ia * 4 + c1) * 4 + c2) * nb + ib]; }
};

// One-site tree a s -> b with factor f: T[ma][c][mb]
struct Tree1 {
  int na, nb;
  std::vector<double> v;
  Tree1(int tja, int s, int tjb, double f) : na(tja + 1), nb(tjb + 1), v(na * 4 * nb, 0.0) {
    for (int ia = 0; ia < na; ++ia)
      for (int u = 0; u <= kLocTJ[s]; ++u)
        for (int ib = 0; ib < nb; ++ib)
          at(ia, kLocC0[s] + u, ib) =
              f * clebsch(tja, tmof(tja, ia), kLocTJ[s], tmof(kLocTJ[s], u), tjb, tmof(tjb, ib));
  }
  double& at(int ia, int c, int ib) { return v[(ia * 4 + c) * nb + ib]; }
  double at(int ia, int c, int ib) const { return v[(ia * 4 + c) * nb + ib]; }
};

// environment coupling Y[m_out][kappa][m_in] = C(j_in m_in; j_w kappa | j_out m_out)
inline double envcg(int tj_in, int i_in, int tjw, int kap, int tj_out, int i_out) {
  return clebsch(tj_in, tmof(tj_in, i_in), tjw, tmof(tjw, kap), tj_out, tmof(tj_out, i_out));
}

inline double sgn_w(int w) { return w == 1 ? 1.0 : -1.0; }
inline double par(int k) { return (k & 1) ? -1.0 : 1.0; }

uint64_t pack(std::initializer_list<int> xs) {
  uint64_t h = 1469598103934665603ull;
  for (int x : xs) {
    h ^= (uint64_t)(uint32_t)(x + 512);
    h *= 1099511628211ull;
  }
  return h;
}

}  // namespace

double Coeffs::onsite2(int s1, int s2) const {
  return onsite1(s1) + onsite1(s2);
}

double Coeffs::onsite1(int s) const {
  // U (n_up-1/2)(n_dn-1/2) is U/4 on the doublet and -U/4 on the singlets
  return s == 0 ? 0.25 * U : -0.25 * U;
}

double Coeffs::left_hop(int site, int w, int tjao, int s1o, int tjai, int s1i, int tjx, int s2, int tjb) {
  uint64_t key = pack({1, site & 1, w, tjao, s1o, tjai, s1i, tjx, s2, tjb});
  auto it = cache.find(key);
  if (it != cache.end()) return it->second * (-t);
  if (!triangle(tjao, kLocTJ[s1o], tjx) || !triangle(tjai, kLocTJ[s1i], tjx)) return 0.0;
  Tree2 to(tjao, s1o, tjx, s2, tjb), ti(tjai, s1i, tjx, s2, tjb);
  SiteOps ops = site_ops(site, 0.0);
  const int tjw = kChTJ[w];
  double acc = 0.0;
  for (int ao = 0; ao <= tjao; ++ao)
    for (int c1o = 0; c1o < 4; ++c1o)
      for (int c2 = 0; c2 < 4; ++c2)
        for (int b = 0; b <= tjb; ++b) {
          double x = to.at(ao, c1o, c2, b);
          if (x == 0.0) continue;
          double y = 0.0;
          for (int ai = 0; ai <= tjai; ++ai)
            for (int c1i = 0; c1i < 4; ++c1i) {
              double th = ti.at(ai, c1i, c2, b);
              if (th == 0.0) continue;
              for (int kap = 0; kap <= tjw; ++kap)
                y += envcg(tjai, ai, tjw, kap, tjao, ao) * ops.right[w][kap][c1o * 4 + c1i] * th;
            }
          acc += x * y;
        }
  double v = par(site - 1) * sgn_w(w) * acc;   // bond (site-1, site)
  cache[key] = v;
  return v * (-t);
}

double Coeffs::right_hop(int site, int w, int tja, int s1, int tjx, int s2o, int tjbo, int s2i, int tjbi) {
  uint64_t key = pack({2, site & 1, w, tja, s1, tjx, s2o, tjbo, s2i, tjbi});
  auto it = cache.find(key);
  if (it != cache.end()) return it->second * (-t);
  if (!triangle(tjx, kLocTJ[s2o], tjbo) || !triangle(tjx, kLocTJ[s2i], tjbi)) return 0.0;
  Tree2 to(tja, s1, tjx, s2o, tjbo), ti(tja, s1, tjx, s2i, tjbi);
  SiteOps ops = site_ops(site + 1, 0.0);
  const int tjw = kChTJ[w];
  double acc = 0.0;
  for (int a = 0; a <= tja; ++a)
    for (int c1 = 0; c1 < 4; ++c1)
      for (int c2o = 0; c2o < 4; ++c2o)
        for (int bo = 0; bo <= tjbo; ++bo) {
          double x = to.at(a, c1, c2o, bo);
          if (x == 0.0) continue;
          double y = 0.0;
          for (int c2i = 0; c2i < 4; ++c2i)
            for (int bi = 0; bi <= tjbi; ++bi) {
              double th = ti.at(a, c1, c2i, bi);
              if (th == 0.0) continue;
              for (int kap = 0; kap <= tjw; ++kap)
                y += ops.left[w][kap][c2o * 4 + c2i] * envcg(tjbi, bi, tjw, kap, tjbo, bo) * th;
            }
          acc += x * y;
        }
  double v = par(site + 1) * sgn_w(w) * acc;   // bond (site+1, site+2)
  cache[key] = v;
  return v * (-t);
}

double Coeffs::mid_hop(int site, int tja, int s1o, int tjxo, int s2o, int s1i, int tjxi, int s2i, int tjb) {
  uint64_t key = pack({3, site & 1, tja, s1o, tjxo, s2o, s1i, tjxi, s2i, tjb});
  auto it = cache.find(key);
  if (it != cache.end()) return it->second * t;
  Tree2 to(tja, s1o, tjxo, s2o, tjb), ti(tja, s1i, tjxi, s2i, tjb);
  Mat16 h = bond_hop(site, 1.0);
  double acc = 0.0;
  for (int a = 0; a <= tja; ++a)
    for (int b = 0; b <= tjb; ++b)
      for (int c1o = 0; c1o < 4; ++c1o)
        for (int c2o = 0; c2o < 4; ++c2o) {
          double x = to.at(a, c1o, c2o, b);
          if (x == 0.0) continue;
          for (int c1i = 0; c1i < 4; ++c1i)
            for (int c2i = 0; c2i < 4; ++c2i) {
              double th = ti.at(a, c1i, c2i, b);
              if (th != 0.0) acc += x * h[(c1o * 4 + c2o) * 16 + (c1i * 4 + c2i)] * th;
            }
        }
  cache[key] = acc;
  return acc * t;
}

double Coeffs::left_hop1(int site, int w, int tjao, int so, int tjai, int si, int tjb) {
  uint64_t key = pack({4, site & 1, w, tjao, so, tjai, si, tjb});
  auto it = cache.find(key);
  if (it != cache.end()) return it->second * (-t);
  Tree1 to(tjao, so, tjb, 1.0 / std::sqrt((double)tjb + 1)), ti(tjai, si, tjb, 1.0 / std::sqrt((double)tjb + 1));
  SiteOps ops = site_ops(site, 0.0);
  const int tjw = kChTJ[w];
  double acc = 0.0;
  for (int ao = 0; ao <= tjao; ++ao)
    for (int co = 0; co < 4; ++co)
      for (int b = 0; b <= tjb; ++b) {
        double x = to.at(ao, co, b);
        if (x == 0.0) continue;
        for (int ai = 0; ai <= tjai; ++ai)
          for (int ci = 0; ci < 4; ++ci) {
            double th = ti.at(ai, ci, b);
            if (th == 0.0) continue;
            for (int kap = 0; kap <= tjw; ++kap)
              acc += x * envcg(tjai, ai, tjw, kap, tjao, ao) * ops.right[w][kap][co * 4 + ci] * th;
          }
      }
  double v = par(site - 1) * sgn_w(w) * acc;
  cache[key] = v;
  return v * (-t);
}

double Coeffs::right_hop1(int site, int w, int tja, int so, int tjbo, int si, int tjbi) {
  uint64_t key = pack({5, site & 1, w, tja, so, tjbo, si, tjbi});
  auto it = cache.find(key);
  if (it != cache.end()) return it->second * (-t);
  Tree1 to(tja, so, tjbo, 1.0 / std::sqrt((double)tjbo + 1)), ti(tja, si, tjbi, 1.0 / std::sqrt((double)tjbi + 1));
  SiteOps ops = site_ops(site, 0.0);
  const int tjw = kChTJ[w];
  double acc = 0.0;
  for (int a = 0; a <= tja; ++a)
    for (int co = 0; co < 4; ++co)
      for (int bo = 0; bo <= tjbo; ++bo) {
        double x = to.at(a, co, bo);
        if (x == 0.0) continue;
        for (int ci = 0; ci < 4; ++ci)
          for (int bi = 0; bi <= tjbi; ++bi) {
            double th = ti.at(a, ci, bi);
            if (th == 0.0) continue;
            for (int kap = 0; kap <= tjw; ++kap)
              acc += x * ops.left[w][kap][co * 4 + ci] * envcg(tjbi, bi, tjw, kap, tjbo, bo) * th;
          }
      }
  double v = par(site) * sgn_w(w) * acc;
  cache[key] = v;
  return v * (-t);
}

double Coeffs::env_left(int site, int wo, int tjbo, int tjbi, int wi, int tjao, int so, int tjai, int si) {
  // E'(b', w', b) += coef A(a',s',b')^dag [E(a', w, a)] A(a, s, b):
  // coef = <Y_out, sum CG(a' s'|b') Op CG(a s|b)> / <Y_out, Y_out>.
  uint64_t key = pack({6, site & 1, wo, tjbo, tjbi, wi, tjao, so, tjai, si});
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  SiteOps ops = site_ops(site, 1.0);   // onsite with U = 1; U applied below
  Tree1 bra(tjao, so, tjbo, 1.0), ket(tjai, si, tjbi, 1.0);
  const int tjwo = wo >= 0 ? kChTJ[wo] : 0;
  double num = 0.0, den = 0.0;
  for (int mo = 0; mo <= tjbo; ++mo)
    for (int kap = 0; kap <= tjwo; ++kap)
      for (int mi = 0; mi <= tjbi; ++mi) {
        double y = envcg(tjbi, mi, tjwo, kap, tjbo, mo);
        if (y == 0.0) continue;
        den += y * y;
        double s = 0.0;
        for (int ao = 0; ao <= tjao; ++ao)
          for (int co = 0; co < 4; ++co) {
            double xb = bra.at(ao, co, mo);
            if (xb == 0.0) continue;
            for (int ai = 0; ai <= tjai; ++ai)
              for (int ci = 0; ci < 4; ++ci) {
                double xk = ket.at(ai, ci, mi);
                if (xk == 0.0) continue;
                double op = 0.0;
                if (wo == 0) {
                  if (wi == 0) op = (ao == ai && co == ci) ? 1.0 : 0.0;
                  else if (wi < 0) op = ao == ai ? U * ops.onsite[co * 4 + ci] : 0.0;
                  else
                    for (int k2 = 0; k2 <= kChTJ[wi]; ++k2)
                      op += -t * par(site - 1) * sgn_w(wi) * envcg(tjai, ai, kChTJ[wi], k2, tjao, ao) *
                            ops.right[wi][k2][co * 4 + ci];
                } else {
                  op = ao == ai ? ops.left[wo][kap][co * 4 + ci] : 0.0;
                }
                s += xb * op * xk;
              }
          }
        num += y * s;
      }
  double v = den > 0 ? num / den : 0.0;
  cache[key] = v;
  return v;
}

double Coeffs::env_right(int site, int wo, int tjxo, int tjxi, int wi, int tjbo, int so, int tjbi, int si) {
  // E'(x', w', x) += coef conj B(x',s',b') [E(b', w, b)] B(x, s, b)^T
  uint64_t key = pack({7, site & 1, wo, tjxo, tjxi, wi, tjbo, so, tjbi, si});
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  SiteOps ops = site_ops(site, 1.0);
  Tree1 bra(tjxo, so, tjbo, std::sqrt((tjxo + 1.0) / (tjbo + 1.0)));
  Tree1 ket(tjxi, si, tjbi, std::sqrt((tjxi + 1.0) / (tjbi + 1.0)));
  const int tjwo = wo >= 0 ? kChTJ[wo] : 0;
  double num = 0.0, den = 0.0;
  for (int mo = 0; mo <= tjxo; ++mo)
    for (int kap = 0; kap <= tjwo; ++kap)
      for (int mi = 0; mi <= tjxi; ++mi) {
        double y = envcg(tjxi, mi, tjwo, kap, tjxo, mo);
        if (y == 0.0) continue;
        den += y * y;
        double s = 0.0;
        for (int co = 0; co < 4; ++co)
          for (int bo = 0; bo <= tjbo; ++bo) {
            double xb = bra.at(mo, co, bo);
            if (xb == 0.0) continue;
            for (int ci = 0; ci < 4; ++ci)
              for (int bi = 0; bi <= tjbi; ++bi) {
                double xk = ket.at(mi, ci, bi);
                if (xk == 0.0) continue;
                double op = 0.0;
                if (wo == 0) {
                  if (wi == 0) op = (bo == bi && co == ci) ? 1.0 : 0.0;
                  else if (wi < 0) op = bo == bi ? U * ops.onsite[co * 4 + ci] : 0.0;
                  else
                    for (int k2 = 0; k2 <= kChTJ[wi]; ++k2)
                      op += -t * par(site) * sgn_w(wi) * ops.left[wi][k2][co * 4 + ci] *
                            envcg(tjbi, bi, kChTJ[wi], k2, tjbo, bo);
                } else {
                  op = bo == bi ? ops.right[wo][kap][co * 4 + ci] : 0.0;
                }
                s += xb * op * xk;
              }
          }
        num += y * s;
      }
  double v = den > 0 ? num / den : 0.0;
  cache[key] = v;
  return v;
}

}  // namespace tdvp

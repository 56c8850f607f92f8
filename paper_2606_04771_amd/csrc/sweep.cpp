// Matrix product state object and the symmetric second-order two-site TDVP
// sweep (supplementary section S2.2: merge two sites, evolve them with the
// Krylov exponential, split by SVD to let the bond grow, evolve the one-site
// centre backwards; truncation by discarded weight, section S2.4).
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <string>
#include <cstring>
#include <map>
#include <memory>
#include <numeric>

#include "device.hpp"
#include "eig.hpp"

using namespace tdvp;

namespace tdvp {

struct Tensor {
  Blocks blk;
  DeviceBuffer buf;
  // Host staging: while `staged`, the data lives in the pinned host buffer
  // `host` (grow-only), the device buffer is given back and blk.data is null.
  void* host = nullptr;
  size_t host_cap = 0;
  bool staged = false;
  ~Tensor() {
    if (host) (void)hipHostFree(host);
  }
};

}  // namespace tdvp

struct tdvp_mps {
  tdvp_ctx* ctx = nullptr;
  tdvp_model model{};
  int L = 0;
  bool fragment = false;   // result of tdvp_split: two sites between open bonds, not a chain
  int sym = 0;             // 0: U(1) x SU(2) sectors (2S^z, 2j); 1: U(1) x U(1) sectors (2S^z, N)
  std::vector<Bond> bonds;                       // 0..L
  std::vector<std::unique_ptr<Tensor>> site;     // site k at index k-1
  std::vector<std::unique_ptr<Tensor>> Lenv, Renv;   // bond 0..L
};

namespace tdvp {

namespace {

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// What the two symmetries differ in, for the chain-level code: the local
// basis (three U(1) x SU(2) multiplets s = 0..2 with charges kLocQ / kLocTJ,
// or four occupation states s = n_up + 2 n_dn with (2S^z, N) = kU1Sz / kU1N),
// the fusion of a bond sector with a local state, the multiplet dimension
// that weights a reduced singular value (2j + 1, or 1) and the block layouts.
constexpr int kU1Sz[4] = {0, 1, -1, 0};
constexpr int kU1N[4] = {0, 1, 1, 2};

inline int nlocal(int sym) { return sym ? 4 : 3; }
inline int64_t multiplet_dim(int sym, int tj) { return sym ? 1 : tj + 1; }

// Does bond sector (q, tj) fused with local state s contain sector (q2, tj2)?
inline bool fuses(int sym, int q, int tj, int s, int q2, int tj2) {
  if (sym) return q + kU1Sz[s] == q2 && tj + kU1N[s] == tj2;
  return q + kLocQ[s] == q2 && triangle(tj, kLocTJ[s], tj2);
}

// Every sector of (q, tj) fused with local state s.
template <class F>
void for_fused(int sym, int q, int tj, int s, F&& f) {
  if (sym) {
    f(q + kU1Sz[s], tj + kU1N[s]);
    return;
  }
  for (int t2 = std::abs(tj - kLocTJ[s]); t2 <= tj + kLocTJ[s]; t2 += 2) f(q + kLocQ[s], t2);
}

int64_t bond_chi(int sym, const Bond& b) { return sym ? b.chi_su2() : b.chi_full(); }

// Two-site blocks: (ia, s1, 2j_x, s2, ib) for U(1) x SU(2), (ia, s1, s2, ib)
// for U(1) x U(1).  The middle sector x and the column pair (s2, ib) of a key.
std::pair<int, int> theta_mid(int sym, const Bond& l, const int* k) {
  if (sym) return {l.q[k[0]] + kU1Sz[k[1]], l.tj[k[0]] + kU1N[k[1]]};
  return {l.q[k[0]] + kLocQ[k[1]], k[2]};
}
std::pair<int, int> theta_col(int sym, const int* k) { return sym ? std::make_pair(k[2], k[3]) : std::make_pair(k[3], k[4]); }

void site_layout(int sym, const Bond& l, const Bond& r, Blocks& out) {
  if (sym) u1_layout_center(l, r, 1, out);
  else layout_site(l, r, out);
}
void theta_layout(int sym, const Bond& l, const Bond& r, Blocks& out) {
  if (sym) u1_layout_center(l, r, 2, out);
  else layout_center(l, r, 2, out);
}

// New contents are about to be written on the device: any staged copy is stale.
int set_site_layout(tdvp_ctx* ctx, Tensor& t, const Bond& l, const Bond& r, int sym) {
  site_layout(sym, l, r, t.blk);
  TDVP_HIP(ctx, t.buf.ensure(sizeof(double) * 2 * (size_t)std::max<int64_t>(t.blk.size, 1)));
  t.blk.data = t.buf.p;
  t.staged = false;
  return TDVP_OK;
}

int set_env_layout(tdvp_ctx* ctx, Tensor& t, const Bond& b, int sym) {
  if (sym) u1_layout_env(b, t.blk);
  else layout_env(b, t.blk);
  TDVP_HIP(ctx, t.buf.ensure(sizeof(double) * 2 * (size_t)std::max<int64_t>(t.blk.size, 1)));
  t.blk.data = t.buf.p;
  t.staged = false;
  return TDVP_OK;
}

// Host staging (paper section S2.3 keeps only the active tensors on the GPU):
// copy a tensor to pinned host memory on the context stream and give its
// device memory back (the allocator orders reuse after the copy: torch's is
// stream-ordered, hipFree waits for the device).
int stage_out(tdvp_ctx* ctx, Tensor& t) {
  if (t.staged || !t.buf.p) return TDVP_OK;
  const size_t bytes = sizeof(double) * 2 * (size_t)std::max<int64_t>(t.blk.size, 1);
  if (t.host_cap < bytes) {
    if (t.host) {   // an earlier copy from this buffer may still be queued
      TDVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
      TDVP_HIP(ctx, hipHostFree(t.host));
      t.host = nullptr;
      t.host_cap = 0;
    }
    TDVP_HIP(ctx, hipHostMalloc(&t.host, bytes));
    t.host_cap = bytes;
  }
  TDVP_HIP(ctx, hipMemcpyAsync(t.host, t.buf.p, bytes, hipMemcpyDeviceToHost, ctx->stream));
  t.buf.release();
  t.blk.data = nullptr;
  t.staged = true;
  return TDVP_OK;
}

// Back to device memory (stream-ordered copy).
int stage_in(tdvp_ctx* ctx, Tensor& t) {
  if (!t.staged) return TDVP_OK;
  const size_t bytes = sizeof(double) * 2 * (size_t)std::max<int64_t>(t.blk.size, 1);
  TDVP_HIP(ctx, t.buf.ensure(bytes));
  TDVP_HIP(ctx, hipMemcpyAsync(t.buf.p, t.host, bytes, hipMemcpyHostToDevice, ctx->stream));
  t.blk.data = t.buf.p;
  t.staged = false;
  return TDVP_OK;
}

// Every tensor of the MPS on the device (calls that read the whole chain).
int unstage_all(tdvp_ctx* ctx, const tdvp_mps* m) {
  for (auto* v : {&m->site, &m->Lenv, &m->Renv})
    for (auto& t : *v)
      if (t)
        if (int rc = stage_in(ctx, *t)) return rc;
  return TDVP_OK;
}

// environment of the empty block (bond [(0,0,1)]): zero Hamiltonian
int empty_env(tdvp_ctx* ctx, Tensor& t, const Bond& b, int sym) {
  int rc = set_env_layout(ctx, t, b, sym);
  if (rc) return rc;
  TDVP_HIP(ctx, hipMemsetAsync(t.blk.data, 0, sizeof(double) * 2 * std::max<int64_t>(t.blk.size, 1), ctx->stream));
  return TDVP_OK;
}

int env_step(tdvp_ctx* ctx, tdvp_mps* m, int site, int dir, double* flops = nullptr) {
  // dir +1: Lenv[site] from Lenv[site-1] and site tensor; -1: Renv[site-1] from Renv[site]
  EnvInputs in;
  in.sym = m->sym;
  if (dir > 0) {
    in.bin = m->bonds[site - 1];
    in.bout = m->bonds[site];
    in.ein = m->Lenv[site - 1]->blk;
    in.ten = m->site[site - 1]->blk;
    int rc = set_env_layout(ctx, *m->Lenv[site], in.bout, m->sym);
    if (rc) return rc;
    in.eout = m->Lenv[site]->blk;
  } else {
    in.bin = m->bonds[site];
    in.bout = m->bonds[site - 1];
    in.ein = m->Renv[site]->blk;
    in.ten = m->site[site - 1]->blk;
    int rc = set_env_layout(ctx, *m->Renv[site - 1], in.bout, m->sym);
    if (rc) return rc;
    in.eout = m->Renv[site - 1]->blk;
  }
  return env_update_dev(ctx, m->model, site, dir, in, flops);
}

int env_step_sync(tdvp_ctx* ctx, tdvp_mps* m, int site, int dir, tdvp_sweep_info* inf) {
  double f = 0.0;
  int rc = env_step(ctx, m, site, dir, &f);
  if (rc) return rc;
  inf->env_flops += f;
  TDVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return TDVP_OK;
}

// Theta(a, s1, x, s2, b) = X(a, s1, x) Y(x, s2, b) for the bond between i and i+1
int merge(tdvp_ctx* ctx, tdvp_mps* m, int i, Blocks& th) {
  const Bond &l = m->bonds[i - 1], &c = m->bonds[i], &r = m->bonds[i + 1];
  theta_layout(m->sym, l, r, th);
  TDVP_HIP(ctx, ctx->ws_theta.ensure(sizeof(double) * 2 * (size_t)std::max<int64_t>(th.size, 1)));
  th.data = ctx->ws_theta.p;
  const Blocks &X = m->site[i - 1]->blk, &Y = m->site[i]->blk;
  auto p = std::make_shared<Program>();
  for (int o = 0; o < th.n(); ++o) {
    const int* k = th.k(o);
    DevOut ob{};
    ob.c_off = th.off[o];
    ob.ldc = ob.M = (int32_t)th.rows[o];
    ob.N = (int32_t)th.cols[o];
    ob.t_begin = (int32_t)p->terms.size();
    const auto x = theta_mid(m->sym, l, k);
    const auto col = theta_col(m->sym, k);
    int ix = c.find(x.first, x.second);
    if (ix >= 0) {
      int a = X.find3(k[0], k[1], ix), b = Y.find3(ix, col.first, col.second);
      if (a >= 0 && b >= 0) {
        DevTerm d{};
        d.coef = 1.0;
        d.a_buf = 0; d.a_off = X.off[a]; d.lda = (int32_t)X.rows[a];
        d.b_buf = 1; d.b_off = Y.off[b]; d.ldb = (int32_t)Y.rows[b];
        d.K = (int32_t)c.d[ix];
        p->terms.push_back(d);
      }
    }
    ob.t_end = ob.d_begin = ob.d_end = (int32_t)p->terms.size();
    p->outs.push_back(ob);
  }
  p->finalize();
  int rc = upload(ctx, *p);
  if (rc) return rc;
  Bufs b{};
  b.p[0] = (const double*)X.data;
  b.p[1] = (const double*)Y.data;
  return launch_gemm(ctx, *p, b, (double*)th.data, TDVP_FP64);
}

struct Sector {
  int q, tj;
  int64_t rows = 0, cols = 0, g = 0;
  std::map<std::pair<int, int>, int64_t> roff, coff;   // (a, s1) -> row, (s2, b) -> col
  int64_t moff = 0, goff = 0, doff = 0;
  bool left_gram = true;   // Gram matrix M M^dag (else M^dag M), always the smaller side
  bool qr = false;         // the isometry lives on the other side: orthonormalise by QR
  int64_t gn = 0;           // padded size of the Gram slot (rows < g hold the eigenvectors)
  int64_t col0 = 0;         // column of the first real eigenvector (n - g padded, 0 unpadded)
  int64_t qoff = 0, iso_off = 0, iso_ld = 0;
  bool scaled = false;      // isometry = M V_k S^-1 without QR
  int keep = 0;
  int64_t iidx = 0;         // slot of the eigensolver's info flag
};

// Batched eigensolver of the sector Gram matrices: divide and conquer on the
// reflected matrices (default), or the Jacobi-based divide and conquer
// directly (TDVP_EIG=jacobi).
bool eig_divide_conquer() {
  static const bool dc = [] {
    const char* e = std::getenv("TDVP_EIG");
    return !(e && std::string(e) == "jacobi");
  }();
  return dc;
}

// Buckets of at least this padded size are solved by the cyclic Jacobi
// eigensolver instead (no tridiagonal reduction: a few launches per sweep
// rather than several per column); read at every split, off by default.
int64_t eig_jacobi_min() {
  const char* e = std::getenv("TDVP_EIG_JACOBI_MIN");
  const long long v = e ? std::atoll(e) : 0;
  return v > 0 ? (int64_t)v : (int64_t)1 << 40;
}

// Buckets of padded size in [this, kTrdMaxN] take the in-house Householder
// tridiagonal reduction (one launch per column for the whole bucket) and the
// library's tridiagonal divide and conquer per matrix, instead of the batched
// library solver; read at every split.
int64_t eig_trd_min() {
  const char* e = std::getenv("TDVP_EIG_TRD_MIN");
  if (!e) return 256;
  const long long v = std::atoll(e);
  return v > 0 ? (int64_t)v : (int64_t)1 << 40;
}

int ensure_solver(tdvp_ctx* ctx) {
  if (ctx->solver) return TDVP_OK;
  rocblas_handle h;
  if (rocblas_create_handle(&h) != rocblas_status_success)
    return set_error(ctx, TDVP_E_HIP, "rocblas_create_handle failed");
  if (rocblas_set_stream(h, ctx->stream) != rocblas_status_success)
    return set_error(ctx, TDVP_E_HIP, "rocblas_set_stream failed");
  ctx->solver = h;
  if (const char* e = std::getenv("TDVP_SIDE_STREAMS")) ctx->nside = std::max(1, std::min(tdvp_ctx::kSide, std::atoi(e)));
  for (int k = 0; k < ctx->nside; ++k) {
    TDVP_HIP(ctx, hipStreamCreateWithFlags(&ctx->side[k], hipStreamNonBlocking));
    rocblas_handle hs;
    if (rocblas_create_handle(&hs) != rocblas_status_success)
      return set_error(ctx, TDVP_E_HIP, "rocblas_create_handle failed");
    ctx->side_solver[k] = hs;
    if (rocblas_set_stream(hs, ctx->side[k]) != rocblas_status_success)
      return set_error(ctx, TDVP_E_HIP, "rocblas_set_stream failed");
  }
  for (auto& ev : ctx->side_ev) TDVP_HIP(ctx, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  // Which side streams share a hardware queue: a 300 us busy wait on stream i,
  // then an event on stream j; if that event completes only after the wait,
  // j's work queues behind i's.  Once per context, ~5 ms.
  for (int j = 0; j < ctx->nside; ++j) {
    ctx->side_group[j] = j;
    for (int i = 0; i < j; ++i) {
      if (ctx->side_group[i] != i) continue;
      if (int r = eig_spin(ctx, ctx->side[i], 300.0)) return r;
      TDVP_HIP(ctx, hipEventRecord(ctx->side_ev[0], ctx->side[i]));
      TDVP_HIP(ctx, hipEventRecord(ctx->side_ev[1], ctx->side[j]));
      TDVP_HIP(ctx, hipEventSynchronize(ctx->side_ev[1]));
      const hipError_t q = hipEventQuery(ctx->side_ev[0]);
      if (q != hipSuccess && q != hipErrorNotReady) TDVP_HIP(ctx, q);
      TDVP_HIP(ctx, hipEventSynchronize(ctx->side_ev[0]));
      if (q == hipSuccess) {
        ctx->side_group[j] = i;
        break;
      }
    }
  }
  if (ctx->verbose) {
    std::string g;
    for (int k = 0; k < ctx->nside; ++k) g += " " + std::to_string(ctx->side_group[k]);
    std::fprintf(stderr, "[tdvp] side streams' hardware-queue groups:%s\n", g.c_str());
  }
  return TDVP_OK;
}

int check_finite(tdvp_ctx* ctx, const Blocks& b, const char* what, int bond);

// Side streams start after the work already on the context stream, and the
// context stream waits for everything then issued on them.
int side_fork(tdvp_ctx* ctx) {
  TDVP_HIP(ctx, hipEventRecord(ctx->side_ev[tdvp_ctx::kSide], ctx->stream));
  for (int k = 0; k < ctx->nside; ++k) TDVP_HIP(ctx, hipStreamWaitEvent(ctx->side[k], ctx->side_ev[tdvp_ctx::kSide], 0));
  return TDVP_OK;
}

int side_join(tdvp_ctx* ctx) {
  for (int k = 0; k < ctx->nside; ++k) {
    TDVP_HIP(ctx, hipEventRecord(ctx->side_ev[k], ctx->side[k]));
    TDVP_HIP(ctx, hipStreamWaitEvent(ctx->stream, ctx->side_ev[k], 0));
  }
  return TDVP_OK;
}

// side stream of each size bucket, largest first, balancing the summed padded size
template <typename Map>
std::vector<int> side_assign(const tdvp_ctx* ctx, const Map& buckets) {
  std::vector<int> who(buckets.size());
  std::vector<double> load(ctx->nside, 0.0);
  int q = (int)buckets.size();
  for (auto it = buckets.rbegin(); it != buckets.rend(); ++it) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[k] += (double)it->first;
    who[--q] = k;
  }
  return who;
}

// Padded sizes for the batched solves.  Every batched call is a chain of
// many small dependent kernels whose length grows with the padded size, so
// fewer, larger buckets beat tight ones: the eigensolves use steps of about
// 1.5x (their calls run concurrently on the side streams), the Cholesky QR of
// the one-site gauge move powers of two (measured at chi = 4096, L = 60).
int64_t bucket_size(int64_t g, bool pow2) {
  static const int64_t eig[] = {1, 2, 4, 8, 16, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048, 3072, 4096};
  if (g > 4096) return (g + 1023) / 1024 * 1024;
  if (pow2) {
    int64_t v = 1;
    while (v < g) v <<= 1;
    return v;
  }
  for (int64_t v : eig)
    if (v >= g) return v;
  return g;
}

int run_program(tdvp_ctx* ctx, Program& p, const Bufs& b, double* C) {
  p.finalize();
  int rc = upload(ctx, p);
  if (!rc) rc = launch_gemm(ctx, p, b, C, TDVP_FP64);
  return rc;
}

// Split Theta at bond i.  dir +1: A_i (left-canonical) and one-site centre on
// site i+1; dir -1: centre on site i and right-canonical B_{i+1}.
//
// Per coupled sector x the block matrix M_x (rows (a, s1), columns (s2, b)) is
// decomposed through the eigenvectors of its smaller Gram matrix (M M^dag or
// M^dag M, dimension g = min(rows, cols)), whose eigenvalues are the squared
// singular values.  That eigenbasis is square, so no part of the range of M
// is lost however small its singular values; when the isometry needed lives on
// the larger side it is obtained by a Householder QR of M V_k (or M^dag U_k).
// The centre is then the exact projection of M on the kept isometry.
int split(tdvp_ctx* ctx, tdvp_mps* m, int i, const Blocks& th, int dir, const tdvp_trunc& tr, double& disc,
          double& t_svd, int& fallbacks, std::vector<double>* svals = nullptr) {
  double t0 = now();
  // phase timestamps (verbose >= 2 only: each one synchronises the stream)
  double ph[4] = {t0, t0, t0, t0};
  auto mark = [&](int k) {
    if (ctx->verbose >= 2 && hipStreamSynchronize(ctx->stream) == hipSuccess) ph[k] = now();
  };
  const Bond &l = m->bonds[i - 1], &r = m->bonds[i + 1];
  const int sym = m->sym, nloc = nlocal(sym);
  std::map<std::pair<int, int>, Sector> secs;
  for (int o = 0; o < th.n(); ++o) {
    const auto x = theta_mid(sym, l, th.k(o));
    Sector& s = secs[x];
    s.q = x.first;
    s.tj = x.second;
  }
  for (auto& kv : secs) {   // every fusion partner of x, in a fixed order
    Sector& s = kv.second;
    for (int a = 0; a < l.size(); ++a)
      for (int s1 = 0; s1 < nloc; ++s1)
        if (fuses(sym, l.q[a], l.tj[a], s1, s.q, s.tj)) {
          s.roff[{a, s1}] = s.rows;
          s.rows += l.d[a];
        }
    for (int s2 = 0; s2 < nloc; ++s2)
      for (int b = 0; b < r.size(); ++b)
        if (fuses(sym, s.q, s.tj, s2, r.q[b], r.tj[b])) {
          s.coff[{s2, b}] = s.cols;
          s.cols += r.d[b];
        }
  }
  // Gram side: always the smaller one (its eigenbasis is square, so no part of
  // range(M) is lost, and it is generically of full rank).  When the isometry
  // lives on the larger side it is M V_k S^-1 (truncation mode, kept singular
  // values far above rounding) or a Householder QR of M V_k (exact mode).
  const bool exact = tr.keep_all || tr.eps_tol < 1e-10;
  std::map<int64_t, std::vector<Sector*>> buckets;   // padded size -> sectors
  for (auto& kv : secs) {
    Sector& s = kv.second;
    s.left_gram = s.rows < s.cols || (s.rows == s.cols && dir > 0);
    s.g = std::min(s.rows, s.cols);
    s.qr = (dir > 0) != s.left_gram;
    if (s.g > 0) buckets[bucket_size(s.g, false)].push_back(&s);
  }
  int64_t mtot = 0, gtot = 0, dtot = 0, nmax = 0, nmat = 0;
  for (auto& kv : secs) {
    Sector& s = kv.second;
    s.moff = mtot;
    mtot += s.rows * s.cols;
  }
  for (auto& bk : buckets) {
    int64_t n = bk.first;
    nmax = std::max(nmax, n);
    for (Sector* s : bk.second) {
      s->gn = n;
      s->goff = gtot;
      gtot += n * n;
      s->doff = dtot;
      dtot += n;
      ++nmat;
    }
  }
  // which buckets the in-house tridiagonal reduction takes, and its storage:
  // reflectors (n^2 complex), tridiagonal eigenvectors (n^2 real), two
  // n-vectors of scratch and the reflector factors (n complex) per matrix
  const bool dc = eig_divide_conquer();
  const int64_t jmin = eig_jacobi_min(), tmin = eig_trd_min();
  // (each of their matrices is reduced at its own size g, not the bucket's
  // padded size; at most kTrdMaxJobs matrices, the largest buckets first)
  const int64_t trd_max = eig_trd_max_n(ctx);
  int64_t trd_lo = std::max<int64_t>(tmin, 1);
  {
    int64_t cnt = 0;
    for (auto it = buckets.rbegin(); it != buckets.rend(); ++it) {
      const int64_t n = it->first;
      if (!(dc && n < jmin && n >= tmin && n <= trd_max)) continue;
      if (cnt + (int64_t)it->second.size() > kTrdMaxJobs) {
        trd_lo = n + 1;
        break;
      }
      cnt += (int64_t)it->second.size();
    }
  }
  auto use_trd = [&](int64_t n) { return dc && n < jmin && n >= trd_lo && n <= trd_max; };
  int64_t tsq = 0, tvec = 0;
  for (auto& bk : buckets)
    if (use_trd(bk.first))
      for (Sector* sp : bk.second) {
        tsq += sp->g * sp->g;
        tvec += sp->g;
      }
  // M | Gram slots | reflector scratch (n complex per slot) | eigenvalues |
  // off-diagonal workspace | Jacobi residuals | info flags | Jacobi sweep
  // counts | tridiagonal-reduction storage
  const size_t tri_bytes = sizeof(double) * (3 * (size_t)tsq + 6 * (size_t)tvec);
  size_t bytes = sizeof(double) * (2 * (size_t)(mtot + gtot) + 2 * (size_t)dtot + 2 * ((size_t)dtot + 8) +
                                   (size_t)(nmat + 8)) +
                 2 * sizeof(rocblas_int) * (size_t)(nmat + 8) + 4096 + 256 + tri_bytes;
  TDVP_HIP(ctx, ctx->ws_svd.ensure(bytes));
  double* Mbase = (double*)ctx->ws_svd.p;
  double* Gbase = Mbase + 2 * mtot;
  double* Pbase = Gbase + 2 * gtot;
  double* Dbase = Pbase + 2 * dtot;
  double* Ebase = Dbase + dtot + 8;
  double* jres = Ebase + dtot + 8;
  rocblas_int* dinfo = (rocblas_int*)(jres + nmat + 8);
  rocblas_int* jsweeps = dinfo + nmat + 8;
  double* tri = (double*)(((uintptr_t)(jsweeps + nmat + 8) + 255) & ~(uintptr_t)255);
  double *triV = tri, *triZ = triV + 2 * tsq, *triY = triZ + tsq, *triT = triY + 4 * tvec;
  int rc;
  Bufs b{};
  // gather Theta blocks into the sector matrices (zeros elsewhere)
  TDVP_HIP(ctx, hipMemsetAsync(Mbase, 0, sizeof(double) * 2 * (size_t)std::max<int64_t>(mtot, 1), ctx->stream));
  {
    Program p;
    for (int o = 0; o < th.n(); ++o) {
      const int* k = th.k(o);
      Sector& s = secs[theta_mid(sym, l, k)];
      DevOut ob{};
      ob.c_off = s.moff + s.roff.at({k[0], k[1]}) + s.coff.at(theta_col(sym, k)) * s.rows;
      ob.ldc = (int32_t)s.rows;
      ob.M = (int32_t)th.rows[o];
      ob.N = (int32_t)th.cols[o];
      ob.t_begin = ob.t_end = ob.d_begin = (int32_t)p.terms.size();
      DevTerm d{};
      d.a_buf = 0; d.a_off = th.off[o]; d.lda = (int32_t)th.rows[o]; d.coef = 1.0;
      p.terms.push_back(d);
      ob.d_end = (int32_t)p.terms.size();
      p.outs.push_back(ob);
    }
    b.p[0] = (const double*)th.data;
    if ((rc = run_program(ctx, p, b, Mbase))) return rc;
  }
  {
    Program g;   // Gram matrices into the leading g x g part of their padded slots
    for (auto& kv : secs) {
      Sector& s = kv.second;
      if (s.g == 0) continue;
      DevOut ob{};
      ob.c_off = s.goff;
      ob.ldc = (int32_t)s.gn;
      ob.M = ob.N = (int32_t)s.g;
      ob.t_begin = (int32_t)g.terms.size();
      DevTerm d{};
      d.coef = 1.0;
      d.a_buf = 0; d.a_off = s.moff; d.lda = (int32_t)s.rows;
      d.b_buf = 0; d.b_off = s.moff; d.ldb = (int32_t)s.rows;
      if (s.left_gram) { d.ops = 4 | 8; d.K = (int32_t)s.cols; }
      else { d.ops = 1 | 2; d.K = (int32_t)s.rows; }
      if (d.K > 0) g.terms.push_back(d);
      ob.t_end = ob.d_begin = ob.d_end = (int32_t)g.terms.size();
      g.outs.push_back(ob);
    }
    b.p[0] = Mbase;
    if ((rc = run_program(ctx, g, b, Gbase))) return rc;
  }
  // padding: negative diagonal entries below every (non-negative) Gram
  // eigenvalue, on the scale of the block's own diagonal
  TDVP_HIP(ctx, ctx->ws_small.ensure(1 << 16));
  {
    double* dscale = (double*)ctx->ws_small.p + 4096;
    int npad = 0;
    for (auto& kv : secs) {
      Sector& s = kv.second;
      if (s.g > 0 && s.g < s.gn) {
        if ((rc = vec_pad_matrix(ctx, Gbase + 2 * s.goff, s.gn, s.g, -1.0, dscale + (npad++ % 1024)))) return rc;
      }
    }
  }
  if ((rc = ensure_solver(ctx))) return rc;
  mark(0);
  auto gram_program = [&](const std::vector<Sector*>& which, Program& g) {
    for (Sector* sp : which) {
      Sector& s = *sp;
      DevOut ob{};
      ob.c_off = s.goff;
      ob.ldc = (int32_t)s.gn;
      ob.M = ob.N = (int32_t)s.g;
      ob.t_begin = (int32_t)g.terms.size();
      DevTerm d{};
      d.coef = 1.0;
      d.a_buf = 0; d.a_off = s.moff; d.lda = (int32_t)s.rows;
      d.b_buf = 0; d.b_off = s.moff; d.ldb = (int32_t)s.rows;
      if (s.left_gram) { d.ops = 4 | 8; d.K = (int32_t)s.cols; }
      else { d.ops = 1 | 2; d.K = (int32_t)s.rows; }
      if (d.K > 0) g.terms.push_back(d);
      ob.t_end = ob.d_begin = ob.d_end = (int32_t)g.terms.size();
      g.outs.push_back(ob);
    }
  };
  {
    // one strided-batched eigensolve per size bucket, the buckets spread over
    // the side streams (largest first) and joined back before verification
    int64_t mi = 0;
    TDVP_HIP(ctx, hipEventRecord(ctx->side_ev[tdvp_ctx::kSide], ctx->stream));
    for (int k = 0; k < ctx->nside; ++k)
      TDVP_HIP(ctx, hipStreamWaitEvent(ctx->side[k], ctx->side_ev[tdvp_ctx::kSide], 0));
    std::vector<std::pair<int64_t, std::vector<Sector*>*>> order;
    for (auto& bk : buckets) order.push_back({bk.first, &bk.second});
    std::vector<int64_t> minfo;
    for (auto& bk : buckets) {
      minfo.push_back(mi);
      mi += (int64_t)bk.second.size();
    }
    // Schedule.  A job is either one batched library solve of a bucket, or
    // (in-house path) one matrix: reflection + reduction, its tridiagonal
    // solve, back-transformation.  The reductions of all in-house matrices
    // share their launches (one per column index, on side stream 0), so a
    // matrix is reduced after as many launches as it has columns; its
    // tridiagonal solve (a chain of small library launches) goes to another
    // hardware queue, waiting for that point by an event, and its
    // back-transformation follows it.  Host issue order: the reductions (then
    // the largest matrix's solve and back-transformation on stream 0), the
    // library solves, then the other tridiagonal solves and
    // back-transformations, so that every event is recorded before a wait on
    // it is issued and the long reduction chain starts first.  Queues are
    // chosen by earliest estimated finish, largest work first.  Issuing from
    // one host thread per stream was measured slower.
    // Cost estimates in milliseconds, fitted to one MI355X (only their ratios
    // steer the schedule): library solve of a bucket, the reduction reaching
    // column n, tridiagonal solve of one matrix, back-transformation.
    auto cost_lib = [](double n, double cnt) { return 0.4 + 0.03 * n + 0.002 * n * (cnt - 1.0); };
    auto cost_stedc = [](double n) { return 0.5 + 0.004 * n; };
    auto cost_back = [](double n, double cnt) { return 0.3 + 8e-4 * n * cnt; };
    struct EigJob {
      int64_t n, cnt, gmax;
      double *G0, *P0, *D0, *E0, *res;
      rocblas_int *info, *sweeps;
      int64_t ld = 0;                 // leading dimension of the matrices (their slot size)
      double *tV = nullptr, *tZ = nullptr, *tY = nullptr, *tT = nullptr;   // tridiagonal-reduction storage
      int home = 0;                   // stream of a library solve / of the back-transformation
      std::vector<int> stedc_on;      // stream of each matrix's tridiagonal solve
      int ev_red = -1;                // event index: reduction done
      std::vector<int> ev_stedc;      // event index per tridiagonal solve off the home stream (-1: home)
    };
    int64_t tsq_at = 0, tvec_at = 0;
    std::vector<EigJob> jobs;         // largest first
    for (int ob = (int)order.size() - 1; ob >= 0; --ob) {
      int64_t n = order[ob].first;
      auto& secv = *order[ob].second;
      Sector* s0 = secv.front();
      int64_t gmax = 0;
      for (size_t q = 0; q < secv.size(); ++q) {
        secv[q]->col0 = n - secv[q]->g;
        secv[q]->iidx = minfo[ob] + (int64_t)q;
        gmax = std::max(gmax, secv[q]->g);
      }
      if (use_trd(n)) {
        // one job per matrix, at its own size (the padding is not touched)
        for (size_t q = 0; q < secv.size(); ++q) {
          Sector* sp = secv[q];
          const int64_t g = sp->g;
          sp->col0 = 0;
          EigJob jb{g, 1, g, Gbase + 2 * sp->goff, Pbase + 2 * sp->doff, Dbase + sp->doff, Ebase + sp->doff,
                    jres + sp->iidx, dinfo + sp->iidx, jsweeps + sp->iidx};
          jb.ld = n;
          jb.tV = triV + 2 * tsq_at;
          jb.tZ = triZ + tsq_at;
          jb.tY = triY + 4 * tvec_at;
          jb.tT = triT + 2 * tvec_at;
          tsq_at += g * g;
          tvec_at += g;
          jobs.push_back(std::move(jb));
        }
        continue;
      }
      EigJob jb{n, (int64_t)secv.size(), gmax, Gbase + 2 * s0->goff, Pbase + 2 * s0->doff,
                Dbase + s0->doff, Ebase + s0->doff, jres + minfo[ob], dinfo + minfo[ob],
                jsweeps + minfo[ob]};
      jb.ld = n;
      jobs.push_back(std::move(jb));
    }
    std::vector<int> trd_ix;          // in-house jobs, smallest first (the order they complete)
    for (int j = 0; j < (int)jobs.size(); ++j)
      if (jobs[j].tV) trd_ix.push_back(j);
    std::stable_sort(trd_ix.begin(), trd_ix.end(), [&](int a, int b) { return jobs[a].n < jobs[b].n; });
    if ((int)trd_ix.size() > kTrdMaxJobs) return set_error(ctx, TDVP_E_INVALID, "too many eigensolver buckets");
    // side stream 0 carries the reductions; the rest take everything else
    // (with one side stream, everything runs on it in issue order)
    const int s_lo = (!trd_ix.empty() && ctx->nside > 1) ? 1 : 0;
    std::vector<double> sfree(ctx->nside, 0.0);
    // (giving the largest matrices' tridiagonal solves streams of their own,
    // the end of the critical path, was measured no faster)
    // streams that share a hardware queue are one resource (sfree is kept on
    // the group's lowest stream); with in-house jobs, stream 0's queue is left
    // to the reductions and their tail when another queue exists
    const int* grp = ctx->side_group;
    bool other_queue = false;
    for (int k = s_lo; k < ctx->nside; ++k) other_queue = other_queue || grp[k] != grp[0];
    auto pick = [&](double ready, double cost) {
      int best = -1;
      for (int k = s_lo; k < ctx->nside; ++k) {
        if (grp[k] != k) continue;   // a group is represented by its lowest stream
        if (s_lo == 1 && other_queue && grp[k] == grp[0]) continue;
        if (best < 0 || std::max(sfree[k], ready) + cost < std::max(sfree[best], ready) + cost) best = k;
      }
      if (best < 0) best = s_lo;
      return best;
    };
    for (EigJob& jb : jobs)
      if (!jb.tV) {
        jb.home = pick(0.0, cost_lib((double)jb.n, (double)jb.cnt));
        sfree[jb.home] += cost_lib((double)jb.n, (double)jb.cnt);
      }
    // when each in-house matrix is reduced: the launches share the trailing
    // matrices' traffic (read and write, ~5 TB/s measured) on top of ~6 us each
    std::vector<double> ready_at(jobs.size(), 0.0);
    {
      double t = 0.0;
      size_t next = 0;
      const int64_t nmax = trd_ix.empty() ? 0 : jobs[trd_ix.back()].n;
      for (int64_t k = 0; k < nmax; ++k) {
        double bytes = 0.0;
        for (size_t q = next; q < trd_ix.size(); ++q) {
          const double m = (double)(jobs[trd_ix[q]].n - k - 1);
          bytes += 32.0 * m * m * (double)jobs[trd_ix[q]].cnt;
        }
        t += 6e-3 + bytes / 5e9;   // ms
        for (; next < trd_ix.size() && jobs[trd_ix[next]].n == k + 1; ++next) ready_at[trd_ix[next]] = t;
      }
      if (!trd_ix.empty()) sfree[0] = std::max(sfree[0], t);
    }
    // The largest matrix is reduced by the last launch: its tridiagonal solve
    // and back-transformation follow the reductions on their stream and are
    // issued right after them, ahead of everything else that may share that
    // stream's hardware queue (sweep 3.81 s; 3.92 s with the solve planned like
    // the others, 3.85 / 4.11 s with the two / three largest on stream 0).
    const int ntail = s_lo == 1 ? std::min<int>(1, (int)trd_ix.size()) : 0;
    int nev = 0;
    for (int j : trd_ix) {
      EigJob& jb = jobs[j];
      const double ready = ready_at[j];
      const bool last = std::find(trd_ix.end() - ntail, trd_ix.end(), j) != trd_ix.end();
      jb.ev_red = nev++;
      double done = ready;
      for (int64_t q = 0; q < jb.cnt; ++q) {
        const int k = last && q == 0 ? 0 : pick(ready, cost_stedc((double)jb.n));
        sfree[k] = std::max(sfree[k], ready) + cost_stedc((double)jb.n);
        done = std::max(done, sfree[k]);
        jb.stedc_on.push_back(k);
      }
      jb.home = jb.stedc_on[0];
      for (int k : jb.stedc_on) jb.ev_stedc.push_back(k == jb.home ? -1 : nev++);
      sfree[jb.home] = std::max(sfree[jb.home], done) + cost_back((double)jb.n, (double)jb.cnt);
    }
    while ((int)ctx->eig_ev.size() < nev) {
      hipEvent_t e;
      TDVP_HIP(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
      ctx->eig_ev.push_back(e);
    }
    // verbose >= 3: a timeline of the phase (start / end of every piece of
    // work against the phase start, "stream:what@start-end" in ms) and the
    // host time spent issuing
    struct Span {
      int stream;
      std::string what;
      hipEvent_t a, b;
    };
    std::vector<Span> spans;
    hipEvent_t t_ref = nullptr;
    if (ctx->verbose >= 3) {
      TDVP_HIP(ctx, hipEventCreate(&t_ref));
      TDVP_HIP(ctx, hipEventRecord(t_ref, ctx->stream));
    }
    auto span_open = [&](int k, const std::string& what) -> int {
      if (!t_ref) return TDVP_OK;
      spans.push_back(Span{k, what, nullptr, nullptr});
      TDVP_HIP(ctx, hipEventCreate(&spans.back().a));
      TDVP_HIP(ctx, hipEventCreate(&spans.back().b));
      TDVP_HIP(ctx, hipEventRecord(spans.back().a, ctx->side[k]));
      return TDVP_OK;
    };
    auto span_close = [&](int k) -> int {
      if (t_ref) TDVP_HIP(ctx, hipEventRecord(spans.back().b, ctx->side[k]));
      return TDVP_OK;
    };
    auto fail = [&](rocblas_status st) {
      return st == rocblas_status_success ? TDVP_OK : set_error(ctx, TDVP_E_HIP, "batched eigensolver failed");
    };
    const double t_issue = now();
    int ec;
    auto issue_trd = [&](int j) -> int {
      const EigJob& jb = jobs[j];
      const int64_t n = jb.n;
      int e2;
      for (int64_t q = 0; q < jb.cnt; ++q) {
        const int k = jb.stedc_on[q];
        TDVP_HIP(ctx, hipStreamWaitEvent(ctx->side[k], ctx->eig_ev[jb.ev_red], 0));
        if ((e2 = span_open(k, "tri" + std::to_string(n)))) return e2;
        if ((e2 = fail(rocsolver_dstedc((rocblas_handle)ctx->side_solver[k], rocblas_evect_tridiagonal,
                                       (rocblas_int)n, jb.D0 + q * n, jb.E0 + q * n, jb.tZ + q * n * n,
                                       (rocblas_int)n, jb.info + q))))
          return e2;
        if ((e2 = span_close(k))) return e2;
        if (jb.ev_stedc[q] >= 0) TDVP_HIP(ctx, hipEventRecord(ctx->eig_ev[jb.ev_stedc[q]], ctx->side[k]));
      }
      const int k = jb.home;
      for (int e : jb.ev_stedc)
        if (e >= 0) TDVP_HIP(ctx, hipStreamWaitEvent(ctx->side[k], ctx->eig_ev[e], 0));
      if ((e2 = span_open(k, "back" + std::to_string(n)))) return e2;
      if ((e2 = eig_trd_back(ctx, ctx->side[k], jb.tZ, jb.tV, jb.tT, jb.G0, n, jb.cnt, n - jb.gmax, jb.ld))) return e2;
      if ((e2 = vec_reflect_back(ctx, ctx->side[k], jb.G0, n, jb.cnt, n - jb.gmax, jb.ld))) return e2;
      return span_close(k);
    };
    // 1. the reductions (the tridiagonal divide and conquer fails on split
    //    tridiagonal forms, so the Gram matrices are reflected first, as for
    //    the library solver below)
    if (!trd_ix.empty()) {
      TrdSet set{};
      int64_t nmax = 0;
      for (int j : trd_ix) {
        EigJob& jb = jobs[j];
        if ((ec = vec_reflect_forward(ctx, ctx->side[0], jb.G0, jb.n, jb.cnt, jb.P0, jb.ld))) return ec;
        set.job[set.njobs++] = TrdJob{jb.G0, jb.tV, jb.tY, jb.tT, jb.D0, jb.E0, (int)jb.n, (int)jb.cnt, (int)jb.ld};
        nmax = std::max(nmax, jb.n);
      }
      TDVP_HIP(ctx, ctx->ws_trd.ensure(sizeof(TrdJob) * kTrdMaxJobs));
      if ((ec = eig_trd_upload(ctx, ctx->side[0], set, ctx->ws_trd.p))) return ec;
      if ((ec = span_open(0, "reduce"))) return ec;
      size_t next = 0;
      for (int64_t k = 0; k < nmax; ++k) {
        if ((ec = eig_trd_column(ctx, ctx->side[0], set, ctx->ws_trd.p, k))) return ec;
        for (; next < trd_ix.size() && jobs[trd_ix[next]].n == k + 1; ++next)
          TDVP_HIP(ctx, hipEventRecord(ctx->eig_ev[jobs[trd_ix[next]].ev_red], ctx->side[0]));
      }
      if ((ec = span_close(0))) return ec;
    }
    // the largest matrices' tridiagonal solves and back-transformations, on
    // stream 0 (largest first), issued before anything else can queue there
    for (int t = 0; t < ntail; ++t)
      if ((ec = issue_trd(trd_ix[trd_ix.size() - 1 - t]))) return ec;
    const double t_issue_red = now();
    // 2. the library solves
    for (const EigJob& jb : jobs) {
      if (jb.tV) continue;
      const int k = jb.home;
      const int64_t n = jb.n;
      if ((ec = span_open(k, "lib" + std::to_string(n) + "x" + std::to_string(jb.cnt)))) return ec;
      if (n >= jmin) {
        // cyclic Jacobi: correct on block-structured and padded matrices as they are
        if ((ec = fail(rocsolver_zheevj_strided_batched(
                 (rocblas_handle)ctx->side_solver[k], rocblas_esort_ascending, rocblas_evect_original,
                 rocblas_fill_upper, (rocblas_int)n, (rocblas_double_complex*)jb.G0, (rocblas_int)n,
                 (rocblas_stride)(n * n), 0.0, jb.res, 100, jb.sweeps, jb.D0, (rocblas_stride)n, jb.info,
                 (rocblas_int)jb.cnt))))
          return ec;
      } else if (dc) {
        // The divide-and-conquer solver returns non-finite eigenvectors when the
        // tridiagonal form splits exactly, which zero-padded or block-structured
        // Gram matrices force; a dense Householder reflection H G H (same
        // spectrum, eigenvectors H W) removes that structure at O(n^2) cost.
        if ((ec = vec_reflect_forward(ctx, ctx->side[k], jb.G0, n, jb.cnt, jb.P0))) return ec;
        if ((ec = fail(rocsolver_zheevd_strided_batched(
                 (rocblas_handle)ctx->side_solver[k], rocblas_evect_original, rocblas_fill_upper, (rocblas_int)n,
                 (rocblas_double_complex*)jb.G0, (rocblas_int)n, (rocblas_stride)(n * n), jb.D0, (rocblas_stride)n,
                 jb.E0, (rocblas_stride)n, jb.info, (rocblas_int)jb.cnt))))
          return ec;
        if ((ec = vec_reflect_back(ctx, ctx->side[k], jb.G0, n, jb.cnt, n - jb.gmax))) return ec;
      } else {
        if ((ec = fail(rocsolver_zheevdj_strided_batched(
                 (rocblas_handle)ctx->side_solver[k], rocblas_evect_original, rocblas_fill_upper, (rocblas_int)n,
                 (rocblas_double_complex*)jb.G0, (rocblas_int)n, (rocblas_stride)(n * n), jb.D0, (rocblas_stride)n,
                 jb.info, (rocblas_int)jb.cnt))))
          return ec;
      }
      if ((ec = span_close(k))) return ec;
    }
    const double t_issue_lib = now();
    // 3. per in-house bucket, in the order the reduction completes them: the
    //    tridiagonal solves, then the eigenvectors of the needed columns
    //    mapped back through both reflections on the home stream (the largest
    //    matrix's were issued right after the reductions)
    for (size_t t = 0; t + ntail < trd_ix.size(); ++t)
      if ((ec = issue_trd(trd_ix[t]))) return ec;
    if (t_ref) {
      const double host_ms = 1e3 * (now() - t_issue);
      TDVP_HIP(ctx, hipDeviceSynchronize());
      std::string line;
      for (Span& x : spans) {
        float a = 0.f, b = 0.f;
        TDVP_HIP(ctx, hipEventElapsedTime(&a, t_ref, x.a));
        TDVP_HIP(ctx, hipEventElapsedTime(&b, t_ref, x.b));
        char buf[128];
        std::snprintf(buf, sizeof buf, " %d:%s@%.1f-%.1f", x.stream, x.what.c_str(), a, b);
        line += buf;
        (void)hipEventDestroy(x.a);
        (void)hipEventDestroy(x.b);
      }
      (void)hipEventDestroy(t_ref);
      std::fprintf(stderr, "[tdvp]   eig bond %d: issue %.2f ms (reductions %.2f, library %.2f);%s\n", i, host_ms,
                   1e3 * (t_issue_red - t_issue), 1e3 * (t_issue_lib - t_issue_red), line.c_str());
    }
    for (int k = 0; k < ctx->nside; ++k) {
      TDVP_HIP(ctx, hipEventRecord(ctx->side_ev[k], ctx->side[k]));
      TDVP_HIP(ctx, hipStreamWaitEvent(ctx->stream, ctx->side_ev[k], 0));
    }
    // verify every bucket's eigenvectors; redo failing buckets unpadded, one matrix at a time
    double* dchk = (double*)ctx->ws_small.p + 2048;
    TDVP_HIP(ctx, ctx->ws_small.ensure(1 << 16));
    dchk = (double*)ctx->ws_small.p + 2048;
    int nb = 0;
    for (auto& bk : buckets) {
      Sector* s0 = bk.second.front();
      if ((rc = vec_norm2(ctx, Gbase + 2 * s0->goff, bk.first * bk.first * (int64_t)bk.second.size(),
                          dchk + 2 * nb)))
        return rc;
      ++nb;
    }
    std::vector<double> chk(2 * std::max(nb, 1));
    std::vector<rocblas_int> binfo(std::max<int64_t>(nmat, 1));
    TDVP_HIP(ctx, hipMemcpyAsync(chk.data(), dchk, sizeof(double) * 2 * nb, hipMemcpyDeviceToHost, ctx->stream));
    TDVP_HIP(ctx, hipMemcpyAsync(binfo.data(), dinfo, sizeof(rocblas_int) * nmat, hipMemcpyDeviceToHost, ctx->stream));
    TDVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    std::vector<Sector*> redo;
    // test hook, read at every split: treat every bucket as failed, so that
    // the unpadded fallback solve is exercised
    const char* ff = std::getenv("TDVP_EIG_FORCE_FALLBACK");
    const bool force_fallback = ff && std::atoi(ff) == 1;
    nb = 0;
    for (auto& bk : buckets) {
      bool bad_info = force_fallback;
      for (Sector* sp : bk.second) bad_info = bad_info || binfo[sp->iidx] != 0;
      if (bad_info || chk[2 * nb + 1] != 0.0 || !std::isfinite(chk[2 * nb])) {
        redo.insert(redo.end(), bk.second.begin(), bk.second.end());
        if (ctx->verbose) {
          std::string gs;
          for (Sector* sp : bk.second) gs += " " + std::to_string(sp->g);
          std::fprintf(stderr, "[tdvp]   bond %d bucket n=%lld failed, g:%s\n", i, (long long)bk.first, gs.c_str());
        }
      }
      ++nb;
    }
    if (!redo.empty()) {
      fallbacks += (int)redo.size();
      if (ctx->verbose) std::fprintf(stderr, "[tdvp]   bond %d: %zu Gram matrices re-solved unpadded\n", i, redo.size());
      Program g;
      gram_program(redo, g);
      b.p[0] = Mbase;
      if ((rc = run_program(ctx, g, b, Gbase))) return rc;
      for (Sector* sp : redo) {
        sp->col0 = 0;
        rocblas_status st = rocsolver_zheevdj((rocblas_handle)ctx->solver, rocblas_evect_original, rocblas_fill_upper,
                                              (rocblas_int)sp->g, (rocblas_double_complex*)(Gbase + 2 * sp->goff),
                                              (rocblas_int)sp->gn, Dbase + sp->doff, dinfo + sp->iidx);
        if (st != rocblas_status_success) return set_error(ctx, TDVP_E_HIP, "rocsolver_zheevdj failed");
      }
    }
  }
  mark(1);
  std::vector<double> ev(std::max<int64_t>(dtot, 1));
  std::vector<rocblas_int> hinfo(std::max<int64_t>(nmat, 1));
  TDVP_HIP(ctx, hipMemcpyAsync(ev.data(), Dbase, sizeof(double) * dtot, hipMemcpyDeviceToHost, ctx->stream));
  TDVP_HIP(ctx, hipMemcpyAsync(hinfo.data(), dinfo, sizeof(rocblas_int) * nmat, hipMemcpyDeviceToHost, ctx->stream));
  TDVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  for (int64_t q = 0; q < nmat; ++q)
    if (hinfo[q] != 0)
      return set_error(ctx, TDVP_E_NOCONV, "eigensolver info " + std::to_string(hinfo[q]) + " at bond " +
                                               std::to_string(i));
  for (auto& kv : secs) {   // the eigenvalues each sector uses (the padding's are not all computed)
    const Sector& s = kv.second;
    for (int64_t q = 0; q < s.g; ++q)
      if (!std::isfinite(ev[s.doff + s.col0 + q]))
        return set_error(ctx, TDVP_E_NONFINITE, "non-finite Gram eigenvalue at bond " + std::to_string(i));
  }
  // truncation: whole multiplets by descending full-state singular value
  struct Ent { double w, sfull; int q, tj, idx; Sector* s; };
  std::vector<Ent> ents;
  double W = 0.0;
  for (auto& kv : secs) {
    Sector& s = kv.second;
    for (int64_t e = 0; e < std::min(s.rows, s.cols); ++e) {   // rank bound
      double lam = std::max(ev[s.doff + s.col0 + s.g - 1 - e], 0.0);   // descending
      ents.push_back({lam, lam / (double)multiplet_dim(sym, s.tj), s.q, s.tj, (int)e, &s});
      W += lam;
    }
  }
  if (!std::isfinite(W)) return set_error(ctx, TDVP_E_NONFINITE, "non-finite singular values");
  if (svals) {   // reduced singular values, sector by sector (ascending (q, 2j)), descending
    svals->clear();
    for (const Ent& e : ents) svals->push_back(std::sqrt(e.w));
  }
  // descending full-state value (sfull is its square); a value closer than
  // 1e-9 of the largest one to its predecessor is a tie, and ties go by
  // (q, 2j) ascending, then position in the sector
  std::stable_sort(ents.begin(), ents.end(), [](const Ent& a, const Ent& b) { return a.sfull > b.sfull; });
  {
    const double tol = ents.empty() ? 0.0 : 1e-9 * std::sqrt(ents[0].sfull);
    size_t g0 = 0;
    for (size_t e = 1; e <= ents.size(); ++e) {
      if (e < ents.size() && std::sqrt(ents[e - 1].sfull) - std::sqrt(ents[e].sfull) <= tol) continue;
      std::stable_sort(ents.begin() + g0, ents.begin() + e, [](const Ent& a, const Ent& b) {
        if (a.q != b.q) return a.q < b.q;
        if (a.tj != b.tj) return a.tj < b.tj;
        return a.idx < b.idx;
      });
      g0 = e;
    }
  }
  size_t keep = ents.size();
  if (!tr.keep_all) {
    double tail = 0.0;
    while (keep > 1 && tail + ents[keep - 1].w <= tr.eps_tol * W) {
      tail += ents[keep - 1].w;
      --keep;
    }
    int64_t chi = 0;
    size_t p = 0;
    for (; p < keep; ++p) {
      if (p > 0 && chi + multiplet_dim(sym, ents[p].tj) > tr.chi_cap) break;
      chi += multiplet_dim(sym, ents[p].tj);
    }
    keep = std::max<size_t>(p, 1);
  }
  double kept = 0.0;
  for (size_t e = 0; e < keep; ++e) {
    ents[e].s->keep++;
    kept += ents[e].w;
  }
  disc = W > 0 ? (W - kept) / W : 0.0;
  double renorm = (!tr.keep_all && kept > 0 && W > 0) ? std::sqrt(W / kept) : 1.0;
  // isometries: eigenvectors directly, or from M V_k / M^dag U_k (scaled, or QR)
  double lam_max = 0.0;
  for (const Ent& e : ents) lam_max = std::max(lam_max, e.w);
  // The scaled isometry M V_k S^-1 is orthonormal up to about
  // eps lam_max / lam_min_kept (the Gram eigensolve's backward error); it is
  // polished by Newton-Schulz steps Q <- Q (3 I - Q^dag Q) / 2, each of which
  // squares that defect, until it is at rounding level.
  double defect = 0.0;
  for (auto& kv : secs) {
    Sector& s = kv.second;
    s.scaled = false;
    if (!s.qr || s.keep == 0 || exact) continue;
    double lam_min_kept = ev[s.doff + s.col0 + s.g - s.keep];
    if (lam_min_kept > 1e-14 * lam_max) {
      s.scaled = true;
      defect = std::max(defect, 2.2e-16 * lam_max / lam_min_kept);
    }
  }
  const int polish = defect > 1e-4 ? 3 : defect > 1e-8 ? 2 : defect > 1e-15 ? 1 : 0;
  int64_t qtot = 0, ktot = 0, kk = 0;
  for (auto& kv : secs) {
    Sector& s = kv.second;
    if (s.keep == 0) continue;
    if (s.qr) {
      int64_t n = dir > 0 ? s.rows : s.cols;
      s.qoff = qtot;
      qtot += n * s.keep;
      ktot += s.keep;
      if (s.scaled) kk += (int64_t)s.keep * s.keep;
      s.iso_off = s.qoff;
      s.iso_ld = n;
    } else {
      s.iso_off = s.goff + (s.col0 + s.g - s.keep) * s.gn;
      s.iso_ld = s.gn;
    }
  }
  const int64_t ptot = polish ? qtot : 0;   // polish scratch: Q^dag Q per sector, Q Q^dag Q
  TDVP_HIP(ctx, ctx->ws_scratch.ensure(sizeof(double) * 2 * (size_t)(qtot + ktot + (polish ? kk : 0) + ptot + 1)));
  double* Qbase = (double*)ctx->ws_scratch.p;
  double* tau = Qbase + 2 * qtot;
  double* Gq = tau + 2 * ktot;
  double* Tq = Gq + 2 * (polish ? kk : 0);
  if (qtot > 0) {
    Program pq;
    for (auto& kv : secs) {
      Sector& s = kv.second;
      if (s.keep == 0 || !s.qr) continue;
      DevOut ob{};
      ob.c_off = s.qoff;
      ob.ldc = ob.M = (int32_t)s.iso_ld;
      ob.N = s.keep;
      ob.t_begin = (int32_t)pq.terms.size();
      DevTerm d{};
      d.coef = 1.0;
      d.a_buf = 0; d.a_off = s.moff; d.lda = (int32_t)s.rows;
      d.b_buf = 1; d.b_off = s.goff + (s.col0 + s.g - s.keep) * s.gn; d.ldb = (int32_t)s.gn;
      if (dir > 0) { d.K = (int32_t)s.cols; d.ops = 0; }       // M V_k
      else { d.K = (int32_t)s.rows; d.ops = 1 | 2; }           // M^dag U_k
      pq.terms.push_back(d);
      ob.t_end = ob.d_begin = ob.d_end = (int32_t)pq.terms.size();
      pq.outs.push_back(ob);
    }
    for (auto& kv : secs) {   // V_k S^-1 (or U_k S^-1) for the scaled projections
      Sector& s = kv.second;
      if (s.keep == 0 || !s.qr || !s.scaled) continue;
      int64_t c0 = s.col0 + s.g - s.keep;
      if ((rc = vec_scale_cols_rsqrt(ctx, Gbase + 2 * (s.goff + c0 * s.gn), s.gn, s.g, s.keep, Dbase + s.doff + c0)))
        return rc;
    }
    b.p[0] = Mbase;
    b.p[1] = Gbase;
    if ((rc = run_program(ctx, pq, b, Qbase))) return rc;
    for (int step = 0; step < polish; ++step) {
      Program pg, pt, pu;   // G = Q^dag Q; T = Q G; Q <- 1.5 Q - 0.5 T
      int64_t go = 0;
      for (auto& kv : secs) {
        Sector& s = kv.second;
        if (s.keep == 0 || !s.qr || !s.scaled) continue;
        const int32_t n = (int32_t)s.iso_ld, k = s.keep;
        DevOut ob{};
        ob.c_off = go;
        ob.ldc = ob.M = ob.N = k;
        ob.t_begin = (int32_t)pg.terms.size();
        DevTerm d{};
        d.coef = 1.0;
        d.a_buf = 0; d.a_off = s.qoff; d.lda = n; d.ops = 1 | 2;
        d.b_buf = 0; d.b_off = s.qoff; d.ldb = n; d.K = n;
        pg.terms.push_back(d);
        ob.t_end = ob.d_begin = ob.d_end = (int32_t)pg.terms.size();
        pg.outs.push_back(ob);
        DevOut ot{};
        ot.c_off = s.qoff;
        ot.ldc = ot.M = n;
        ot.N = k;
        ot.t_begin = (int32_t)pt.terms.size();
        DevTerm e{};
        e.coef = 1.0;
        e.a_buf = 0; e.a_off = s.qoff; e.lda = n;
        e.b_buf = 1; e.b_off = go; e.ldb = k; e.K = k;
        pt.terms.push_back(e);
        ot.t_end = ot.d_begin = ot.d_end = (int32_t)pt.terms.size();
        pt.outs.push_back(ot);
        DevOut ou{};
        ou.c_off = s.qoff;
        ou.ldc = ou.M = n;
        ou.N = k;
        ou.t_begin = ou.t_end = ou.d_begin = (int32_t)pu.terms.size();
        DevTerm u1{}, u2{};
        u1.a_buf = 0; u1.a_off = s.qoff; u1.lda = n; u1.coef = 1.5;
        u2.a_buf = 1; u2.a_off = s.qoff; u2.lda = n; u2.coef = -0.5;
        pu.terms.push_back(u1);
        pu.terms.push_back(u2);
        ou.d_end = (int32_t)pu.terms.size();
        pu.outs.push_back(ou);
        go += (int64_t)k * k;
      }
      Bufs bq{};
      bq.p[0] = Qbase;
      if ((rc = run_program(ctx, pg, bq, Gq))) return rc;
      bq.p[1] = Gq;
      if ((rc = run_program(ctx, pt, bq, Tq))) return rc;
      bq.p[1] = Tq;   // element-wise, in place: every output element reads only its own inputs
      if ((rc = run_program(ctx, pu, bq, Qbase))) return rc;
    }
    int64_t kofs = 0;
    for (auto& kv : secs) {
      Sector& s = kv.second;
      if (s.keep == 0 || !s.qr || s.scaled) continue;
      auto* A = (rocblas_double_complex*)(Qbase + 2 * s.qoff);
      auto* tq = (rocblas_double_complex*)(tau + 2 * kofs);
      kofs += s.keep;
      rocblas_status st = rocsolver_zgeqrf((rocblas_handle)ctx->solver, (rocblas_int)s.iso_ld, s.keep, A,
                                           (rocblas_int)s.iso_ld, tq);
      if (st == rocblas_status_success)
        st = rocsolver_zungqr((rocblas_handle)ctx->solver, (rocblas_int)s.iso_ld, s.keep, s.keep, A,
                              (rocblas_int)s.iso_ld, tq);
      if (st != rocblas_status_success) return set_error(ctx, TDVP_E_HIP, "rocsolver QR failed");
    }
  }
  mark(2);
  // new bond i
  Bond nb;
  for (auto& kv : secs)
    if (kv.second.keep > 0) nb.add(kv.second.q, kv.second.tj, kv.second.keep);
  m->bonds[i] = nb;
  Tensor& TA = *m->site[i - 1];
  Tensor& TB = *m->site[i];
  rc = set_site_layout(ctx, TA, m->bonds[i - 1], nb, sym);
  if (!rc) rc = set_site_layout(ctx, TB, nb, m->bonds[i + 1], sym);
  if (rc) return rc;
  // buffers: 0 = eigenvectors (Gbase), 1 = M, 2 = QR isometries
  auto iso_buf = [](const Sector& s) { return s.qr ? 2 : 0; };
  Program pa, pb;
  auto sector_of = [&](int ix) -> Sector& { return secs[{nb.q[ix], nb.tj[ix]}]; };
  if (dir > 0) {
    for (int o = 0; o < TA.blk.n(); ++o) {   // A(a, s1, x) = U_k rows (a, s1)
      const int* k = TA.blk.k(o);
      Sector& s = sector_of(k[2]);
      DevOut ob{};
      ob.c_off = TA.blk.off[o];
      ob.ldc = ob.M = (int32_t)TA.blk.rows[o];
      ob.N = (int32_t)TA.blk.cols[o];
      ob.t_begin = ob.t_end = ob.d_begin = (int32_t)pa.terms.size();
      DevTerm d{};
      d.a_buf = iso_buf(s); d.a_off = s.iso_off + s.roff.at({k[0], k[1]}); d.lda = (int32_t)s.iso_ld;
      d.coef = 1.0;
      pa.terms.push_back(d);
      ob.d_end = (int32_t)pa.terms.size();
      pa.outs.push_back(ob);
    }
    for (int o = 0; o < TB.blk.n(); ++o) {   // C(x, s2, b) = U_k^dag M[:, (s2, b)]
      const int* k = TB.blk.k(o);
      Sector& s = sector_of(k[0]);
      DevOut ob{};
      ob.c_off = TB.blk.off[o];
      ob.ldc = ob.M = (int32_t)TB.blk.rows[o];
      ob.N = (int32_t)TB.blk.cols[o];
      ob.t_begin = (int32_t)pb.terms.size();
      DevTerm d{};
      d.coef = renorm;
      d.a_buf = iso_buf(s); d.a_off = s.iso_off; d.lda = (int32_t)s.iso_ld; d.ops = 1 | 2;
      d.b_buf = 1; d.b_off = s.moff + s.coff.at({k[1], k[2]}) * s.rows; d.ldb = (int32_t)s.rows;
      d.K = (int32_t)s.rows;
      pb.terms.push_back(d);
      ob.t_end = ob.d_begin = ob.d_end = (int32_t)pb.terms.size();
      pb.outs.push_back(ob);
    }
  } else {
    for (int o = 0; o < TA.blk.n(); ++o) {   // C(a, s1, x) = M[(a, s1), :] V_k
      const int* k = TA.blk.k(o);
      Sector& s = sector_of(k[2]);
      DevOut ob{};
      ob.c_off = TA.blk.off[o];
      ob.ldc = ob.M = (int32_t)TA.blk.rows[o];
      ob.N = (int32_t)TA.blk.cols[o];
      ob.t_begin = (int32_t)pa.terms.size();
      DevTerm d{};
      d.coef = renorm;
      d.a_buf = 1; d.a_off = s.moff + s.roff.at({k[0], k[1]}); d.lda = (int32_t)s.rows;
      d.b_buf = iso_buf(s); d.b_off = s.iso_off; d.ldb = (int32_t)s.iso_ld;
      d.K = (int32_t)s.cols;
      pa.terms.push_back(d);
      ob.t_end = ob.d_begin = ob.d_end = (int32_t)pa.terms.size();
      pa.outs.push_back(ob);
    }
    for (int o = 0; o < TB.blk.n(); ++o) {   // B(x, s2, b) = (V_k[(s2, b), :])^dag
      const int* k = TB.blk.k(o);
      Sector& s = sector_of(k[0]);
      DevOut ob{};
      ob.c_off = TB.blk.off[o];
      ob.ldc = ob.M = (int32_t)TB.blk.rows[o];
      ob.N = (int32_t)TB.blk.cols[o];
      ob.t_begin = ob.t_end = ob.d_begin = (int32_t)pb.terms.size();
      DevTerm d{};
      d.a_buf = iso_buf(s); d.a_off = s.iso_off + s.coff.at({k[1], k[2]}); d.lda = (int32_t)s.iso_ld;
      d.ops = 1 | 2;
      d.coef = 1.0;
      pb.terms.push_back(d);
      ob.d_end = (int32_t)pb.terms.size();
      pb.outs.push_back(ob);
    }
  }
  b.p[0] = Gbase;
  b.p[1] = Mbase;
  b.p[2] = Qbase;
  if ((rc = run_program(ctx, pa, b, (double*)TA.blk.data))) return rc;
  if ((rc = run_program(ctx, pb, b, (double*)TB.blk.data))) return rc;
  TDVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  t_svd += now() - t0;
  if (ctx->verbose >= 2) {
    std::string bs;
    for (auto& bk : buckets) bs += " " + std::to_string(bk.first) + "x" + std::to_string(bk.second.size());
    std::fprintf(stderr, "[tdvp]   split bond %d: gram %.4f eig %.4f iso %.4f out %.4f s (%zu sectors, %lld matrices;%s)\n",
                 i, ph[0] - t0, ph[1] - ph[0], ph[2] - ph[1], now() - ph[2], secs.size(), (long long)nmat, bs.c_str());
  }
  return TDVP_OK;
}

int evolve(tdvp_ctx* ctx, tdvp_mps* m, int site, int nsites, Blocks& x, const Blocks& Le, const Blocks& Re,
           double tau_im, const tdvp_trunc& tr, tdvp_sweep_info* info) {
  HeffInputs in;
  in.sym = m->sym;
  in.l = m->bonds[site - 1];
  in.r = m->bonds[site + nsites - 1];
  in.Le = Le;
  in.Re = Re;
  in.x = x;
  KrylovResult kr;
  int rc = krylov_dev(ctx, m->model, site, nsites, in, {0.0, tau_im}, tr.krylov_tol, tr.krylov_maxdim, kr);
  info->krylov_iters += kr.iters;
  info->graph_iters += kr.graph_iters;
  info->krylov_max = std::max(info->krylov_max, kr.iters);
  info->heff_flops += kr.heff_flops;
  if (rc == TDVP_E_NOCONV) {
    info->nonconverged++;
    rc = TDVP_OK;
  }
  return rc;
}

// debug aid (verbose >= 2): fail with a named phase when a tensor is not finite
int check_finite(tdvp_ctx* ctx, const Blocks& b, const char* what, int bond) {
  if (ctx->verbose < 2 || b.size == 0) return TDVP_OK;
  TDVP_HIP(ctx, ctx->ws_small.ensure(1 << 16));
  double* d = (double*)ctx->ws_small.p + 1024;
  int rc = vec_norm2(ctx, (const double*)b.data, b.size, d);
  if (rc) return rc;
  double h[2];
  TDVP_HIP(ctx, hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
  TDVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  std::fprintf(stderr, "[tdvp]   check %-10s bond %2d |x|^2=%.6e nonfinite=%.0f\n", what, bond, h[0], h[1]);
  if (h[1] != 0.0 || !std::isfinite(h[0]))
    return set_error(ctx, TDVP_E_NONFINITE, std::string("non-finite ") + what + " at bond " + std::to_string(bond));
  return TDVP_OK;
}

int build_right_envs(tdvp_ctx* ctx, tdvp_mps* m) {
  int L = m->L;
  int rc = empty_env(ctx, *m->Renv[L], m->bonds[L], m->sym);
  if (rc) return rc;
  for (int k = L; k >= 2; --k)
    if ((rc = env_step(ctx, m, k, -1))) return rc;
  return empty_env(ctx, *m->Lenv[0], m->bonds[0], m->sym);
}

tdvp_mps* new_mps(tdvp_ctx* ctx, const tdvp_model& model) {
  auto* m = new tdvp_mps();
  m->ctx = ctx;
  m->model = model;
  m->L = model.L;
  m->bonds.resize(m->L + 1);
  for (int k = 0; k < m->L; ++k) m->site.emplace_back(new Tensor());
  for (int k = 0; k <= m->L; ++k) {
    m->Lenv.emplace_back(new Tensor());
    m->Renv.emplace_back(new Tensor());
  }
  for (auto* v : {&m->site, &m->Lenv, &m->Renv})
    for (auto& t : *v) t->buf.al = ctx->alloc;
  return m;
}

// Sector counts of a block of n sites: multiplets per (2S^z, 2j) (sym 0) or
// states per (2S^z, N) (sym 1).
std::map<std::pair<int, int>, int64_t> sector_counts(int sym, int n) {
  std::map<std::pair<int, int>, int64_t> cur{{{0, 0}, 1}};
  for (int s = 0; s < n; ++s) {
    std::map<std::pair<int, int>, int64_t> nxt;
    for (auto& kv : cur)
      for (int l = 0; l < nlocal(sym); ++l)
        for_fused(sym, kv.first.first, kv.first.second, l, [&](int q, int tj) { nxt[{q, tj}] += kv.second; });
    cur.swap(nxt);
  }
  return cur;
}

// The Neel product state (up on odd sites) at half filling, right-canonical
// with the centre on site 1; with `complete`, every bond at the full
// dimension its sectors can have in the chain (zero-weight directions kept).
int create_neel(tdvp_ctx* ctx, const tdvp_model* model, int32_t complete, int sym, tdvp_mps** out) {
  if (!ctx || !model || !out) return set_error(ctx, TDVP_E_INVALID, "null argument");
  return guarded(ctx, [&]() -> int {
    *out = nullptr;
    const int L = model->L;
    if (L < 2 || L % 2) return set_error(ctx, TDVP_E_INVALID, "the Neel state needs an even L >= 2");
    TDVP_HIP(ctx, hipSetDevice(ctx->device));
    std::unique_ptr<tdvp_mps> m(new_mps(ctx, *model));
    m->sym = sym;
    auto neel_s = [](int k) { return (k & 1) ? 1 : 2; };   // up on odd sites
    // sector of the Neel state's first k sites, and the partner a right block
    // of L - k sites needs for the whole chain to be the Neel state's sector
    // (2S^z = 0; pseudospin singlet, or N = L)
    auto neel_label = [&](int k) { return sym ? std::make_pair(k & 1, k) : std::make_pair(k & 1, 0); };
    auto partner = [&](int q, int tj) { return sym ? std::make_pair(-q, L - tj) : std::make_pair(-q, tj); };
    // bond sectors
    std::vector<std::map<std::pair<int, int>, int64_t>> mult(L + 1);
    for (int n = 0; n <= L; ++n) mult[n] = sector_counts(sym, n);
    for (int k = 0; k <= L; ++k) {
      Bond b;
      if (complete) {
        for (auto& kv : mult[k]) {
          auto it = mult[L - k].find(partner(kv.first.first, kv.first.second));
          if (it == mult[L - k].end()) continue;
          b.add(kv.first.first, kv.first.second, std::min(kv.second, it->second));
        }
      } else {
        b.add(neel_label(k).first, neel_label(k).second, 1);
      }
      m->bonds[k] = b;
    }
    // right-canonical tensors by selecting rows of the identity on the fused
    // space, always keeping the Neel path; centre on site 1 selects the Neel path
    std::vector<int64_t> neel_idx(L + 1, 0);
    std::vector<std::vector<double>> host(L);
    for (int k = L; k >= 1; --k) {
      Tensor& T = *m->site[k - 1];
      int rc = set_site_layout(ctx, T, m->bonds[k - 1], m->bonds[k], sym);
      if (rc) return rc;
      const Bond &l = m->bonds[k - 1], &r = m->bonds[k];
      host[k - 1].assign(2 * (size_t)T.blk.size, 0.0);
      int ia_neel = l.find(neel_label(k - 1).first, neel_label(k - 1).second);
      int ib_neel = r.find(neel_label(k).first, neel_label(k).second);
      for (int ia = 0; ia < l.size(); ++ia) {
        // columns of the fused space for row sector ia, in block order
        std::vector<int> blocks;
        int64_t F = 0;
        std::vector<int64_t> coff;
        for (int o = 0; o < T.blk.n(); ++o)
          if (T.blk.k(o)[0] == ia) {
            blocks.push_back(o);
            coff.push_back(F);
            F += T.blk.cols[o];
          }
        int64_t d = l.d[ia];
        int64_t pos_neel = -1;
        if (ia == ia_neel)
          for (size_t j = 0; j < blocks.size(); ++j) {
            const int* kk = T.blk.k(blocks[j]);
            if (kk[1] == neel_s(k) && kk[2] == ib_neel) pos_neel = coff[j] + neel_idx[k];
          }
        if (k == 1) {   // centre: only the Neel entry
          for (size_t j = 0; j < blocks.size(); ++j) {
            const int* kk = T.blk.k(blocks[j]);
            if (ia == ia_neel && kk[1] == neel_s(k) && kk[2] == ib_neel)
              host[0][2 * (T.blk.off[blocks[j]] + 0 + neel_idx[1] * T.blk.rows[blocks[j]])] = 1.0;
          }
          continue;
        }
        std::vector<int64_t> sel;
        if (pos_neel >= 0) sel.push_back(pos_neel);
        for (int64_t c = 0; (int64_t)sel.size() < d && c < F; ++c)
          if (c != pos_neel) sel.push_back(c);
        std::sort(sel.begin(), sel.end());
        if ((int64_t)sel.size() != d) return set_error(ctx, TDVP_E_SHAPE, "inconsistent complete bond dimensions");
        if (pos_neel >= 0)
          neel_idx[k - 1] = std::lower_bound(sel.begin(), sel.end(), pos_neel) - sel.begin();
        for (int64_t rr = 0; rr < d; ++rr) {
          int64_t c = sel[rr];
          size_t j = std::upper_bound(coff.begin(), coff.end(), c) - coff.begin() - 1;
          int o = blocks[j];
          int64_t cc = c - coff[j];
          host[k - 1][2 * (T.blk.off[o] + rr + cc * T.blk.rows[o])] = 1.0;
        }
      }
    }
    for (int k = 1; k <= L; ++k)
      TDVP_HIP(ctx, hipMemcpy(m->site[k - 1]->blk.data, host[k - 1].data(), sizeof(double) * host[k - 1].size(),
                              hipMemcpyHostToDevice));
    int rc = build_right_envs(ctx, m.get());
    if (rc) return rc;
    TDVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *out = m.release();
    return TDVP_OK;
  });
}

// An MPS from caller blocks (right-canonical, centre on site 1).
int create_from_blocks(tdvp_ctx* ctx, const tdvp_model* model, const tdvp_bond* bonds, const tdvp_blocks* sites,
                       int sym, tdvp_mps** out) {
  if (!ctx || !model || !out || !bonds || !sites) return set_error(ctx, TDVP_E_INVALID, "null argument");
  return guarded(ctx, [&]() -> int {
    *out = nullptr;
    if (model->L < 2) return set_error(ctx, TDVP_E_INVALID, "L must be >= 2");
    TDVP_HIP(ctx, hipSetDevice(ctx->device));
    std::unique_ptr<tdvp_mps> m(new_mps(ctx, *model));
    m->sym = sym;
    std::string err;
    for (int k = 0; k <= m->L; ++k) {
      int rc = sym ? u1_load_bond(m->bonds[k], &bonds[k], err) : load_bond(m->bonds[k], &bonds[k], err);
      if (rc) return set_error(ctx, rc, err);
    }
    const Bond &b0 = m->bonds[0], &bL = m->bonds[m->L];
    if (b0.size() != 1 || b0.q[0] != 0 || b0.tj[0] != 0 || b0.d[0] != 1)
      return set_error(ctx, TDVP_E_SECTOR, "bond 0 must be the single sector (0,0) of dimension 1");
    // U(1) x SU(2): the chain is a pseudospin singlet with S^z = 0; U(1) x U(1):
    // the last bond's one sector is the chain's (2S^z, N)
    if (bL.size() != 1 || bL.d[0] != 1 || (!sym && (bL.q[0] != 0 || bL.tj[0] != 0)))
      return set_error(ctx, TDVP_E_SECTOR,
                       sym ? "bond L must be a single sector of dimension 1"
                           : "boundary bonds must be the single sector (0,0) of dimension 1");
    for (int k = 1; k <= m->L; ++k) {
      Blocks src;
      int rc = sym ? u1_load_center(src, &sites[k - 1], m->bonds[k - 1], m->bonds[k], 1, err)
                   : load_site(src, &sites[k - 1], m->bonds[k - 1], m->bonds[k], err);
      if (rc) return set_error(ctx, rc, err);
      if (src.n() && !src.data) return set_error(ctx, TDVP_E_INVALID, "null device data");
      rc = set_site_layout(ctx, *m->site[k - 1], m->bonds[k - 1], m->bonds[k], sym);
      if (rc) return rc;
      TDVP_HIP(ctx, hipMemsetAsync(m->site[k - 1]->blk.data, 0,
                                   sizeof(double) * 2 * std::max<int64_t>(m->site[k - 1]->blk.size, 1), ctx->stream));
      rc = copy_blocks(ctx, src, m->site[k - 1]->blk, 1.0);
      if (rc) return rc;
    }
    int rc = build_right_envs(ctx, m.get());
    if (rc) return rc;
    TDVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *out = m.release();
    return TDVP_OK;
  });
}

}  // namespace

}  // namespace tdvp

extern "C" {

int tdvp_mps_create_neel(tdvp_ctx* ctx, const tdvp_model* model, int32_t complete, tdvp_mps** out) {
  return create_neel(ctx, model, complete, 0, out);
}

int tdvp_u1_mps_create_neel(tdvp_ctx* ctx, const tdvp_model* model, int32_t complete, tdvp_mps** out) {
  return create_neel(ctx, model, complete, 1, out);
}

int tdvp_mps_create(tdvp_ctx* ctx, const tdvp_model* model, const tdvp_bond* bonds, const tdvp_blocks* sites,
                    tdvp_mps** out) {
  return create_from_blocks(ctx, model, bonds, sites, 0, out);
}

int tdvp_u1_mps_create(tdvp_ctx* ctx, const tdvp_model* model, const tdvp_bond* bonds, const tdvp_blocks* sites,
                       tdvp_mps** out) {
  return create_from_blocks(ctx, model, bonds, sites, 1, out);
}

void tdvp_mps_destroy(tdvp_mps* mps) {
  // The owning context may already be gone: do not touch it.  Device memory
  // goes back to the context's allocator after outstanding work has finished.
  if (!mps) return;
  (void)hipDeviceSynchronize();
  delete mps;
}

int tdvp_mps_bond(const tdvp_mps* m, int32_t k, int32_t* n, int32_t* q, int32_t* tj, int64_t* dim) {
  if (!m || !n || k < 0 || k > m->L) return set_error(nullptr, TDVP_E_INVALID, "bad arguments");
  const Bond& b = m->bonds[k];
  *n = b.size();
  for (int i = 0; i < b.size(); ++i) {
    if (q) q[i] = b.q[i];
    if (tj) tj[i] = b.tj[i];
    if (dim) dim[i] = b.d[i];
  }
  return TDVP_OK;
}

int tdvp_mps_site_layout(const tdvp_mps* m, int32_t k, int32_t* nblocks, int32_t* keys, int64_t* offsets,
                         int64_t* total) {
  if (!m || !nblocks || k < 1 || k > m->L) return set_error(nullptr, TDVP_E_INVALID, "bad arguments");
  const Blocks& b = m->site[k - 1]->blk;
  *nblocks = b.n();
  if (total) *total = b.size;
  if (keys) std::memcpy(keys, b.key.data(), sizeof(int) * b.key.size());
  if (offsets) std::memcpy(offsets, b.off.data(), sizeof(int64_t) * b.off.size());
  return TDVP_OK;
}

int tdvp_mps_site_read(tdvp_ctx* ctx, const tdvp_mps* m, int32_t k, void* host_dst) {
  if (!ctx || !m || !host_dst || k < 1 || k > m->L) return set_error(ctx, TDVP_E_INVALID, "bad arguments");
  if (int rc = stage_in(ctx, *m->site[k - 1])) return rc;
  const Blocks& b = m->site[k - 1]->blk;
  TDVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  TDVP_HIP(ctx, hipMemcpy(host_dst, b.data, sizeof(double) * 2 * b.size, hipMemcpyDeviceToHost));
  return TDVP_OK;
}

int tdvp_sweep(tdvp_ctx* ctx, tdvp_mps* m, double dt, const tdvp_trunc* tr, tdvp_sweep_info* info) {
  if (!ctx || !m || !tr) return set_error(ctx, TDVP_E_INVALID, "null argument");
  return guarded(ctx, [&]() -> int {
    if (m->ctx != ctx) return set_error(ctx, TDVP_E_INVALID, "MPS belongs to another context");
    if (m->fragment) return set_error(ctx, TDVP_E_INVALID, "a split result is not a chain");
    if (tr->krylov_maxdim < 1 || tr->krylov_maxdim > 64) return set_error(ctx, TDVP_E_INVALID, "bad krylov_maxdim");
    TDVP_HIP(ctx, hipSetDevice(ctx->device));
    tdvp_sweep_info inf{};
    double t0 = now();
    const int L = m->L;
    const double tau = 0.5 * dt;
    int rc;
    Blocks th;
    auto timed = [&](double& acc, auto&& f) -> int {
      double s = now();
      int r = f();
      acc += now() - s;
      return r;
    };
    auto vlog = [&](const char* dirs, int i, double tb, const tdvp_sweep_info& a, const tdvp_sweep_info& b,
                    int64_t n) {
      if (!ctx->verbose) return;
      std::fprintf(stderr,
                   "[tdvp] %s bond %2d chi=%6lld theta=%9lld krylov=%3d t=%.3fs (lanczos %.3f svd %.3f env %.3f)\n",
                   dirs, i, (long long)bond_chi(m->sym, m->bonds[i]), (long long)n, b.krylov_iters - a.krylov_iters,
                   now() - tb, b.t_lanczos - a.t_lanczos, b.t_svd - a.t_svd, b.t_env - a.t_env);
      std::fflush(stderr);
    };
    // host staging: the tensors of the bond being updated come to the device
    // before it, and those the next bond does not read go back to host memory
    // after it (a left-to-right step leaves L_{i-1}, R_{i+1} and A_i behind,
    // a right-to-left one R_{i+1}, L_{i-1} and B_{i+1})
    const bool staging = ctx->host_staging;
    auto bring = [&](int i) -> int {
      if (!staging) return TDVP_OK;
      for (Tensor* t : {m->Lenv[i - 1].get(), m->Renv[i + 1].get(), m->site[i - 1].get(), m->site[i].get()})
        if (int r = stage_in(ctx, *t)) return r;
      return TDVP_OK;
    };
    auto park = [&](std::initializer_list<Tensor*> ts) -> int {
      if (!staging) return TDVP_OK;
      for (Tensor* t : ts)
        if (int r = stage_out(ctx, *t)) return r;
      return TDVP_OK;
    };
    for (int i = 1; i <= L - 1; ++i) {
      double tb = now();
      tdvp_sweep_info before = inf;
      if ((rc = bring(i))) return rc;
      if ((rc = merge(ctx, m, i, th))) return rc;
      if ((rc = check_finite(ctx, th, "merge", i))) return rc;
      if ((rc = timed(inf.t_lanczos, [&] {
             return evolve(ctx, m, i, 2, th, m->Lenv[i - 1]->blk, m->Renv[i + 1]->blk, -tau, *tr, &inf);
           })))
        return rc;
      if ((rc = check_finite(ctx, th, "evolved", i))) return rc;
      double d = 0;
      if ((rc = split(ctx, m, i, th, +1, *tr, d, inf.t_svd, inf.eig_fallbacks))) return rc;
      if ((rc = check_finite(ctx, m->site[i - 1]->blk, "split-A", i))) return rc;
      if ((rc = check_finite(ctx, m->site[i]->blk, "split-C", i))) return rc;
      inf.max_discarded = std::max(inf.max_discarded, d);
      inf.sum_discarded += d;
      if ((rc = timed(inf.t_env, [&] { return env_step_sync(ctx, m, i, +1, &inf); })))
        return rc;
      if ((rc = check_finite(ctx, m->Lenv[i]->blk, "Lenv", i))) return rc;
      if (i < L - 1) {
        Blocks& c = m->site[i]->blk;
        if ((rc = timed(inf.t_lanczos, [&] {
               return evolve(ctx, m, i + 1, 1, c, m->Lenv[i]->blk, m->Renv[i + 1]->blk, +tau, *tr, &inf);
             })))
          return rc;
      }
      if (i < L - 1 && (rc = park({m->Lenv[i - 1].get(), m->Renv[i + 1].get(), m->site[i - 1].get()}))) return rc;
      vlog("L->R", i, tb, before, inf, th.size);
    }
    for (int i = L - 1; i >= 1; --i) {
      double tb = now();
      tdvp_sweep_info before = inf;
      if ((rc = bring(i))) return rc;
      if ((rc = merge(ctx, m, i, th))) return rc;
      if ((rc = timed(inf.t_lanczos, [&] {
             return evolve(ctx, m, i, 2, th, m->Lenv[i - 1]->blk, m->Renv[i + 1]->blk, -tau, *tr, &inf);
           })))
        return rc;
      double d = 0;
      if ((rc = split(ctx, m, i, th, -1, *tr, d, inf.t_svd, inf.eig_fallbacks))) return rc;
      inf.max_discarded = std::max(inf.max_discarded, d);
      inf.sum_discarded += d;
      if ((rc = timed(inf.t_env, [&] { return env_step_sync(ctx, m, i + 1, -1, &inf); })))
        return rc;
      if (i > 1) {
        Blocks& c = m->site[i - 1]->blk;
        if ((rc = timed(inf.t_lanczos, [&] {
               return evolve(ctx, m, i, 1, c, m->Lenv[i - 1]->blk, m->Renv[i]->blk, +tau, *tr, &inf);
             })))
          return rc;
      }
      if (i > 1 && (rc = park({m->Renv[i + 1].get(), m->Lenv[i - 1].get(), m->site[i].get()}))) return rc;
      vlog("R->L", i, tb, before, inf, th.size);
    }
    TDVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int k = 0; k <= L; ++k) {
      inf.max_chi = std::max(inf.max_chi, bond_chi(m->sym, m->bonds[k]));
      inf.max_chi_su2 = std::max(inf.max_chi_su2, m->bonds[k].chi_su2());
    }
    {
      bool bad = false;
      if ((rc = take_bad_flag(ctx, bad))) return rc;
      if (bad) return set_error(ctx, TDVP_E_NONFINITE, "non-finite values during the sweep");
    }
    inf.seconds = now() - t0;
    if (info) *info = inf;
    return TDVP_OK;
  });
}

}  // extern "C"

// Local observables of the state C_1 B_2 ... B_L (centre on site 1, the rest
// right-canonical).  The overlap environment N_k[b] of bond k (one matrix per
// sector, the full-state one being N_k[b] (x) 1) obeys
//   N_k[b] = sum_{a,s} (2j_a+1)/(2j_b+1) T[a,s,b]^dag N_{k-1}[a] T[a,s,b]
// for both the centre and the B tensors (the centre's left bond is the
// vacuum), and the weight of local multiplet s on site k is
//   W_s(k) = sum_{a,b} (2j_a+1) tr(T[a,s,b]^dag N_{k-1}[a] T[a,s,b]).
// S^z is +1/2 on |up>, -1/2 on |down>, 0 on the doublet; in a pseudospin
// singlet the doublet weight splits evenly between |up,down> and |0>.  For a
// U(1) x U(1) chain the dimension factors are 1 and s runs over the four
// occupation states, |up,down> being s = 3.
int tdvp_mps_measure(tdvp_ctx* ctx, const tdvp_mps* m, double* sz, double* docc, double* norm2) {
  if (!ctx || !m || !sz || !docc) return set_error(ctx, TDVP_E_INVALID, "null argument");
  return guarded(ctx, [&]() -> int {
    if (m->ctx != ctx) return set_error(ctx, TDVP_E_INVALID, "MPS belongs to another context");
    if (m->fragment) return set_error(ctx, TDVP_E_INVALID, "a split result is not a chain");
    TDVP_HIP(ctx, hipSetDevice(ctx->device));
    const int L = m->L;
    int rc;
    if ((rc = unstage_all(ctx, m))) return rc;
    // sector-diagonal layout of N on bond k
    auto nlayout = [](const Bond& b, Blocks& nb) {
      nb = Blocks();
      nb.keylen = 1;
      int64_t o = 0;
      for (int i = 0; i < b.size(); ++i) {
        int key = i;
        nb.push(&key, o, b.d[i], b.d[i]);
        o += b.d[i] * b.d[i];
      }
      nb.size = o;
    };
    int64_t nmax = 1, tmax = 1, bmax = 1;
    for (int k = 0; k <= L; ++k) {
      int64_t s = 0;
      for (int i = 0; i < m->bonds[k].size(); ++i) s += m->bonds[k].d[i] * m->bonds[k].d[i];
      nmax = std::max(nmax, s);
    }
    for (int k = 1; k <= L; ++k) {
      tmax = std::max(tmax, m->site[k - 1]->blk.size);
      bmax = std::max<int64_t>(bmax, m->site[k - 1]->blk.n());
    }
    DeviceBuffer nbuf[2], t1, meta, part;
    use_alloc(ctx, {&nbuf[0], &nbuf[1], &t1, &meta, &part});
    TDVP_HIP(ctx, nbuf[0].ensure(sizeof(double) * 2 * nmax));
    TDVP_HIP(ctx, nbuf[1].ensure(sizeof(double) * 2 * nmax));
    TDVP_HIP(ctx, t1.ensure(sizeof(double) * 2 * tmax));
    TDVP_HIP(ctx, meta.ensure(sizeof(int64_t) * 2 * bmax));
    TDVP_HIP(ctx, part.ensure(sizeof(double) * 2 * bmax));
    // N_0: identity on every sector of bond 0
    Blocks Nin, Nout;
    nlayout(m->bonds[0], Nin);
    {
      std::vector<double> h(2 * (size_t)Nin.size, 0.0);
      for (int i = 0; i < Nin.n(); ++i)
        for (int64_t r = 0; r < Nin.rows[i]; ++r) h[2 * (Nin.off[i] + r + r * Nin.rows[i])] = 1.0;
      TDVP_HIP(ctx, hipMemcpyAsync(nbuf[0].p, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice,
                                   ctx->stream));
      TDVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }
    int cur = 0;
    double last_norm = 0.0;
    std::vector<double> hp(2 * bmax);
    std::vector<int64_t> hm(2 * bmax);
    for (int k = 1; k <= L; ++k) {
      const Blocks& T = m->site[k - 1]->blk;
      const Bond &l = m->bonds[k - 1], &r = m->bonds[k];
      nlayout(r, Nout);
      Program p1, p2;
      for (int o = 0; o < T.n(); ++o) {   // T1 = N[a] . T[a, s, b]
        const int* key = T.k(o);
        DevOut ob{};
        ob.c_off = T.off[o];
        ob.ldc = ob.M = (int32_t)T.rows[o];
        ob.N = (int32_t)T.cols[o];
        ob.t_begin = (int32_t)p1.terms.size();
        DevTerm d{};
        d.coef = 1.0;
        d.a_buf = 0; d.a_off = Nin.off[key[0]]; d.lda = (int32_t)Nin.rows[key[0]];
        d.b_buf = 1; d.b_off = T.off[o]; d.ldb = (int32_t)T.rows[o];
        d.K = (int32_t)T.rows[o];
        p1.terms.push_back(d);
        ob.t_end = ob.d_begin = ob.d_end = (int32_t)p1.terms.size();
        p1.outs.push_back(ob);
      }
      for (int b = 0; b < r.size(); ++b) {   // N'[b] = sum c T^dag T1
        DevOut ob{};
        ob.c_off = Nout.off[b];
        ob.ldc = ob.M = ob.N = (int32_t)r.d[b];
        ob.t_begin = (int32_t)p2.terms.size();
        for (int o = 0; o < T.n(); ++o) {
          const int* key = T.k(o);
          if (key[2] != b) continue;
          DevTerm d{};
          d.coef = (double)multiplet_dim(m->sym, l.tj[key[0]]) / (double)multiplet_dim(m->sym, r.tj[b]);
          d.a_buf = 1; d.a_off = T.off[o]; d.lda = (int32_t)T.rows[o]; d.ops = 1 | 2;
          d.b_buf = 2; d.b_off = T.off[o]; d.ldb = (int32_t)T.rows[o];
          d.K = (int32_t)T.rows[o];
          p2.terms.push_back(d);
        }
        ob.t_end = ob.d_begin = ob.d_end = (int32_t)p2.terms.size();
        p2.outs.push_back(ob);
      }
      Bufs bf{};
      bf.p[0] = (const double*)nbuf[cur].p;
      bf.p[1] = (const double*)T.data;
      bf.p[2] = (const double*)t1.p;
      if ((rc = run_program(ctx, p1, bf, (double*)t1.p))) return rc;
      if ((rc = run_program(ctx, p2, bf, (double*)nbuf[1 - cur].p))) return rc;
      for (int o = 0; o < T.n(); ++o) {
        hm[2 * o] = T.off[o];
        hm[2 * o + 1] = T.rows[o] * T.cols[o];
      }
      TDVP_HIP(ctx, hipMemcpyAsync(meta.p, hm.data(), sizeof(int64_t) * 2 * T.n(), hipMemcpyHostToDevice,
                                   ctx->stream));
      if ((rc = vec_block_dots(ctx, (const double*)T.data, (const double*)t1.p, (const int64_t*)meta.p, T.n(),
                               (double*)part.p)))
        return rc;
      TDVP_HIP(ctx, hipMemcpyAsync(hp.data(), part.p, sizeof(double) * 2 * T.n(), hipMemcpyDeviceToHost,
                                   ctx->stream));
      TDVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
      double W[4] = {0.0, 0.0, 0.0, 0.0};
      for (int o = 0; o < T.n(); ++o) {
        const int* key = T.k(o);
        W[key[1]] += (double)multiplet_dim(m->sym, l.tj[key[0]]) * hp[2 * o];
      }
      const double nrm = W[0] + W[1] + W[2] + W[3];
      if (!std::isfinite(nrm) || nrm <= 0.0)
        return set_error(ctx, TDVP_E_NONFINITE, "state norm not positive and finite at site " + std::to_string(k));
      // |up> and |down> are s = 1, 2 in both local bases; the double occupancy
      // is half the pseudospin doublet's weight (s = 0) or the weight of s = 3
      sz[k - 1] = 0.5 * (W[1] - W[2]) / nrm;
      docc[k - 1] = (m->sym ? W[3] : 0.5 * W[0]) / nrm;
      last_norm = nrm;
      Nin = Nout;
      cur = 1 - cur;
    }
    if (norm2) *norm2 = last_norm;
    return TDVP_OK;
  });
}

// <bra|ket> of two MPS on the same chain (any gauge, bond dimensions may
// differ): the mixed overlap environment on bond k, one d_bra x d_ket matrix
// per sector present in both, obeys
//   N_k[b] = sum_{a,s} (2j_a+1)/(2j_b+1) bra[a,s,b]^dag N_{k-1}[a] ket[a,s,b]
// (the same recoupling as the norm; factors 1 for U(1) x U(1)), and
// <bra|ket> = N_L on the last bond's one sector.
int tdvp_mps_overlap(tdvp_ctx* ctx, const tdvp_mps* bra, const tdvp_mps* ket, double* out) {
  if (!ctx || !bra || !ket || !out) return set_error(ctx, TDVP_E_INVALID, "null argument");
  return guarded(ctx, [&]() -> int {
    if (bra->ctx->device != ctx->device || ket->ctx->device != ctx->device)
      return set_error(ctx, TDVP_E_INVALID, "MPS on another device");
    if (bra->L != ket->L) return set_error(ctx, TDVP_E_SHAPE, "chains of different length");
    if (bra->sym != ket->sym) return set_error(ctx, TDVP_E_INVALID, "chains of different symmetry");
    if (bra->fragment || ket->fragment) return set_error(ctx, TDVP_E_INVALID, "a split result is not a chain");
    TDVP_HIP(ctx, hipSetDevice(ctx->device));
    if (int r0 = unstage_all(ctx, bra)) return r0;
    if (int r0 = unstage_all(ctx, ket)) return r0;
    const int L = ket->L;
    int rc;
    // environment layout on bond k: blocks keyed by the ket's sector index
    struct Env {
      Blocks blk;
      std::vector<int> bra_ix;   // bra sector of each block
    };
    auto layout = [&](int k, Env& e) {
      e.blk = Blocks();
      e.blk.keylen = 1;
      e.bra_ix.clear();
      const Bond &bb = bra->bonds[k], &kb = ket->bonds[k];
      int64_t o = 0;
      for (int i = 0; i < kb.size(); ++i) {
        int j = bb.find(kb.q[i], kb.tj[i]);
        if (j < 0) continue;
        e.blk.push(&i, o, bb.d[j], kb.d[i]);
        e.bra_ix.push_back(j);
        o += bb.d[j] * kb.d[i];
      }
      e.blk.size = o;
    };
    int64_t nmax = 1, tmax = 1;
    for (int k = 0; k <= L; ++k) {
      Env e;
      layout(k, e);
      nmax = std::max(nmax, e.blk.size);
    }
    for (int k = 1; k <= L; ++k) {
      const Blocks& T = ket->site[k - 1]->blk;
      const Bond& lb = bra->bonds[k - 1];
      int64_t s = 0;
      for (int o = 0; o < T.n(); ++o) {
        int j = lb.find(ket->bonds[k - 1].q[T.k(o)[0]], ket->bonds[k - 1].tj[T.k(o)[0]]);
        if (j >= 0) s += lb.d[j] * T.cols[o];
      }
      tmax = std::max(tmax, s);
    }
    DeviceBuffer nbuf[2], t1;
    use_alloc(ctx, {&nbuf[0], &nbuf[1], &t1});
    TDVP_HIP(ctx, nbuf[0].ensure(sizeof(double) * 2 * nmax));
    TDVP_HIP(ctx, nbuf[1].ensure(sizeof(double) * 2 * nmax));
    TDVP_HIP(ctx, t1.ensure(sizeof(double) * 2 * tmax));
    Env Nin, Nout;
    layout(0, Nin);
    {
      std::vector<double> h(2 * (size_t)std::max<int64_t>(Nin.blk.size, 1), 0.0);
      for (int i = 0; i < Nin.blk.n(); ++i)
        for (int64_t r = 0; r < std::min(Nin.blk.rows[i], Nin.blk.cols[i]); ++r)
          h[2 * (Nin.blk.off[i] + r + r * Nin.blk.rows[i])] = 1.0;
      TDVP_HIP(ctx, hipMemcpyAsync(nbuf[0].p, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice,
                                   ctx->stream));
      TDVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }
    int cur = 0;
    for (int k = 1; k <= L; ++k) {
      const Blocks &K = ket->site[k - 1]->blk, &B = bra->site[k - 1]->blk;
      const Bond &kl = ket->bonds[k - 1], &kr = ket->bonds[k];
      const Bond &bl = bra->bonds[k - 1], &br = bra->bonds[k];
      layout(k, Nout);
      // stage 1: T1[o] = N[a] . ket[o] for ket blocks whose left sector is common
      Program p1, p2;
      std::vector<int64_t> t1off(K.n(), -1);
      int64_t to = 0;
      std::map<int, int> nin_of;   // ket sector -> Nin block
      for (int i = 0; i < Nin.blk.n(); ++i) nin_of[Nin.blk.k(i)[0]] = i;
      for (int o = 0; o < K.n(); ++o) {
        const int* key = K.k(o);
        auto it = nin_of.find(key[0]);
        if (it == nin_of.end()) continue;
        const int ni = it->second;
        t1off[o] = to;
        DevOut ob{};
        ob.c_off = to;
        ob.ldc = ob.M = (int32_t)Nin.blk.rows[ni];
        ob.N = (int32_t)K.cols[o];
        ob.t_begin = (int32_t)p1.terms.size();
        DevTerm d{};
        d.coef = 1.0;
        d.a_buf = 0; d.a_off = Nin.blk.off[ni]; d.lda = (int32_t)Nin.blk.rows[ni];
        d.b_buf = 1; d.b_off = K.off[o]; d.ldb = (int32_t)K.rows[o];
        d.K = (int32_t)K.rows[o];
        p1.terms.push_back(d);
        ob.t_end = ob.d_begin = ob.d_end = (int32_t)p1.terms.size();
        p1.outs.push_back(ob);
        to += Nin.blk.rows[ni] * K.cols[o];
      }
      // stage 2: Nout[b] = sum c bra[a', s, b']^dag T1[o]
      for (int i = 0; i < Nout.blk.n(); ++i) {
        const int kb = Nout.blk.k(i)[0], bb = Nout.bra_ix[i];
        DevOut ob{};
        ob.c_off = Nout.blk.off[i];
        ob.ldc = ob.M = (int32_t)br.d[bb];
        ob.N = (int32_t)kr.d[kb];
        ob.t_begin = (int32_t)p2.terms.size();
        for (int o = 0; o < K.n(); ++o) {
          const int* key = K.k(o);
          if (key[2] != kb || t1off[o] < 0) continue;
          int ba = bl.find(kl.q[key[0]], kl.tj[key[0]]);
          int bo = B.find3(ba, key[1], bb);
          if (bo < 0) continue;
          DevTerm d{};
          d.coef = (double)multiplet_dim(ket->sym, kl.tj[key[0]]) / (double)multiplet_dim(ket->sym, kr.tj[kb]);
          d.a_buf = 2; d.a_off = B.off[bo]; d.lda = (int32_t)B.rows[bo]; d.ops = 1 | 2;
          d.b_buf = 3; d.b_off = t1off[o]; d.ldb = (int32_t)B.rows[bo];
          d.K = (int32_t)B.rows[bo];
          p2.terms.push_back(d);
        }
        ob.t_end = ob.d_begin = ob.d_end = (int32_t)p2.terms.size();
        p2.outs.push_back(ob);
      }
      Bufs bf{};
      bf.p[0] = (const double*)nbuf[cur].p;
      bf.p[1] = (const double*)K.data;
      bf.p[2] = (const double*)B.data;
      bf.p[3] = (const double*)t1.p;
      if ((rc = run_program(ctx, p1, bf, (double*)t1.p))) return rc;
      if ((rc = run_program(ctx, p2, bf, (double*)nbuf[1 - cur].p))) return rc;
      Nin = Nout;
      cur = 1 - cur;
    }
    double h[2] = {0.0, 0.0};
    if (Nin.blk.n() == 1 && Nin.blk.rows[0] == 1 && Nin.blk.cols[0] == 1)
      TDVP_HIP(ctx, hipMemcpyAsync(h, nbuf[cur].p, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    TDVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    out[0] = h[0];
    out[1] = h[1];
    return TDVP_OK;
  });
}

// ---------------------------------------------------------------------------
// One-site TDVP (supplementary section S2.2: once the bond dimension has
// saturated, the single-site projector splitting needs no SVD; the centre
// moves by a QR of the one-site tensor and the bond matrix is evolved
// backwards with the zero-site effective Hamiltonian).
namespace tdvp {
namespace {

// One square block per sector of bond b (the bond matrix), contiguous.
void bondmat_layout(const Bond& b, Blocks& x) {
  x = Blocks();
  x.keylen = 1;
  int64_t o = 0;
  for (int i = 0; i < b.size(); ++i) {
    int key = i;
    x.push(&key, o, b.d[i], b.d[i]);
    o += b.d[i] * b.d[i];
  }
  x.size = o;
}

// The sector (of the bond being cut) that block o of a one-site tensor belongs to.
inline int cut_sector(const Blocks& T, int o, int dir) { return dir > 0 ? T.k(o)[2] : T.k(o)[0]; }

// Gauge move of the one-site tensor T at site i by QR (dir +1: T = A x on bond
// i, A left-canonical) or LQ (dir -1: T = x B on bond i-1, B right-canonical),
// sector by sector of the cut bond, with the bond dimensions unchanged.
// CholeskyQR2: G = M^dag M per sector (grouped GEMM), G = R^dag R (batched
// Cholesky), Q1 = M R^-1 (batched triangular inverse + grouped GEMM), and
// the same once more on Q1, which restores orthogonality to rounding for
// condition numbers up to ~1e7.  A bond whose Cholesky fails (rank-deficient
// centre, e.g. complete bases) is done by Householder QR per sector instead.
// On return T holds A (or B) and xbuf the bond matrix (layout bondmat_layout).
int gauge_qr(tdvp_ctx* ctx, tdvp_mps* m, int i, int dir, Blocks& x, DeviceBuffer& xbuf, DeviceBuffer& qbuf) {
  Tensor& TT = *m->site[i - 1];
  Blocks& T = TT.blk;
  const Bond& cut = dir > 0 ? m->bonds[i] : m->bonds[i - 1];
  bondmat_layout(cut, x);
  TDVP_HIP(ctx, xbuf.ensure(sizeof(double) * 2 * (size_t)std::max<int64_t>(x.size, 1)));
  x.data = xbuf.p;
  TDVP_HIP(ctx, qbuf.ensure(sizeof(double) * 2 * (size_t)std::max<int64_t>(T.size, 1)));
  int rc;
  if ((rc = ensure_solver(ctx))) return rc;
  const int ns = cut.size();
  // padded Gram slots by size bucket
  std::vector<int64_t> gn(ns), goff(ns);
  std::map<int64_t, std::vector<int>> buckets;
  for (int s = 0; s < ns; ++s) buckets[bucket_size(cut.d[s], true)].push_back(s);
  int64_t gtot = 0;
  for (auto& bk : buckets)
    for (int s : bk.second) {
      gn[s] = bk.first;
      goff[s] = gtot;
      gtot += bk.first * bk.first;
    }
  // regions: G (work), R1, R2 (kept), info
  size_t bytes = sizeof(double) * 2 * (size_t)(3 * gtot) + sizeof(rocblas_int) * (size_t)(ns + 8) + 4096;
  TDVP_HIP(ctx, ctx->ws_svd.ensure(bytes));
  double* G = (double*)ctx->ws_svd.p;
  double* R1 = G + 2 * gtot;
  double* R2 = R1 + 2 * gtot;
  rocblas_int* dinfo = (rocblas_int*)(R2 + 2 * gtot);
  Bufs b{};
  // one CholeskyQR round on the tensor in buffer src (layout of T) into dst; R kept in Rk
  auto round = [&](const double* src, double* dst, double* Rk) -> int {
    TDVP_HIP(ctx, hipMemsetAsync(G, 0, sizeof(double) * 2 * (size_t)gtot, ctx->stream));
    Program pg;
    for (int s = 0; s < ns; ++s) {
      DevOut ob{};
      ob.c_off = goff[s];
      ob.ldc = (int32_t)gn[s];
      ob.M = ob.N = (int32_t)cut.d[s];
      ob.t_begin = (int32_t)pg.terms.size();
      for (int o = 0; o < T.n(); ++o) {
        if (cut_sector(T, o, dir) != s) continue;
        DevTerm d{};
        d.coef = 1.0;
        d.a_buf = 0; d.a_off = T.off[o]; d.lda = (int32_t)T.rows[o];
        d.b_buf = 0; d.b_off = T.off[o]; d.ldb = (int32_t)T.rows[o];
        if (dir > 0) { d.ops = 1 | 2; d.K = (int32_t)T.rows[o]; }   // M^dag M over rows (a, s)
        else { d.ops = 4 | 8; d.K = (int32_t)T.cols[o]; }           // M M^dag over columns (s, b)
        pg.terms.push_back(d);
      }
      ob.t_end = ob.d_begin = ob.d_end = (int32_t)pg.terms.size();
      pg.outs.push_back(ob);
    }
    b.p[0] = src;
    int r;
    if ((r = run_program(ctx, pg, b, G))) return r;
    for (int s = 0; s < ns; ++s)
      if ((r = vec_pad_identity(ctx, G + 2 * goff[s], gn[s], cut.d[s]))) return r;
    // batched Cholesky per size bucket, the buckets spread over the side streams
    const std::vector<int> who = side_assign(ctx, buckets);
    if ((r = side_fork(ctx))) return r;
    int64_t mi = 0;
    int q = 0;
    for (auto& bk : buckets) {
      const int64_t n = bk.first;
      const int s0 = bk.second.front(), cnt = (int)bk.second.size();
      rocblas_status st = rocsolver_zpotrf_strided_batched(
          (rocblas_handle)ctx->side_solver[who[q++]], rocblas_fill_upper, (rocblas_int)n,
          (rocblas_double_complex*)(G + 2 * goff[s0]), (rocblas_int)n, (rocblas_stride)(n * n), dinfo + mi, cnt);
      if (st != rocblas_status_success) return set_error(ctx, TDVP_E_HIP, "rocsolver_zpotrf_strided_batched failed");
      mi += cnt;
    }
    if ((r = side_join(ctx))) return r;
    std::vector<rocblas_int> info(ns);
    TDVP_HIP(ctx, hipMemcpyAsync(info.data(), dinfo, sizeof(rocblas_int) * ns, hipMemcpyDeviceToHost, ctx->stream));
    TDVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int q = 0; q < ns; ++q)
      if (info[q] != 0) return TDVP_E_NOCONV;   // not positive definite to working precision
    // keep R (upper), then invert it in place in G
    TDVP_HIP(ctx, hipMemcpyAsync(Rk, G, sizeof(double) * 2 * (size_t)gtot, hipMemcpyDeviceToDevice, ctx->stream));
    for (auto& bk : buckets) {
      const int64_t n = bk.first;
      const int s0 = bk.second.front(), cnt = (int)bk.second.size();
      if ((r = vec_zero_lower(ctx, Rk + 2 * goff[s0], n, cnt))) return r;
      if ((r = vec_zero_lower(ctx, G + 2 * goff[s0], n, cnt))) return r;
    }
    if ((r = side_fork(ctx))) return r;
    q = 0;
    mi = 0;
    for (auto& bk : buckets) {
      const int64_t n = bk.first;
      const int s0 = bk.second.front(), cnt = (int)bk.second.size();
      rocblas_status st = rocsolver_ztrtri_strided_batched(
          (rocblas_handle)ctx->side_solver[who[q++]], rocblas_fill_upper, rocblas_diagonal_non_unit, (rocblas_int)n,
          (rocblas_double_complex*)(G + 2 * goff[s0]), (rocblas_int)n, (rocblas_stride)(n * n), dinfo + mi, cnt);
      if (st != rocblas_status_success) return set_error(ctx, TDVP_E_HIP, "rocsolver_ztrtri_strided_batched failed");
      mi += cnt;
    }
    if ((r = side_join(ctx))) return r;
    // dst = src R^-1 (dir +1) or R^-dag src (dir -1), block by block
    Program pq;
    for (int o = 0; o < T.n(); ++o) {
      const int s = cut_sector(T, o, dir);
      DevOut ob{};
      ob.c_off = T.off[o];
      ob.ldc = ob.M = (int32_t)T.rows[o];
      ob.N = (int32_t)T.cols[o];
      ob.t_begin = (int32_t)pq.terms.size();
      DevTerm d{};
      d.coef = 1.0;
      if (dir > 0) {
        d.a_buf = 0; d.a_off = T.off[o]; d.lda = (int32_t)T.rows[o];
        d.b_buf = 1; d.b_off = goff[s]; d.ldb = (int32_t)gn[s];
        d.K = (int32_t)cut.d[s];
      } else {
        d.a_buf = 1; d.a_off = goff[s]; d.lda = (int32_t)gn[s]; d.ops = 1 | 2;
        d.b_buf = 0; d.b_off = T.off[o]; d.ldb = (int32_t)T.rows[o];
        d.K = (int32_t)cut.d[s];
      }
      pq.terms.push_back(d);
      ob.t_end = ob.d_begin = ob.d_end = (int32_t)pq.terms.size();
      pq.outs.push_back(ob);
    }
    b.p[0] = src;
    b.p[1] = G;
    return run_program(ctx, pq, b, dst);
  };
  double* Q1 = (double*)qbuf.p;
  rc = round((const double*)T.data, Q1, R1);
  if (!rc) rc = round(Q1, (double*)T.data, R2);
  if (rc == TDVP_OK) {
    // x = R2 R1 (dir +1) or (R2 R1)^dag = R1^dag R2^dag (dir -1)
    Program px;
    for (int s = 0; s < ns; ++s) {
      DevOut ob{};
      ob.c_off = x.off[s];
      ob.ldc = ob.M = ob.N = (int32_t)cut.d[s];
      ob.t_begin = (int32_t)px.terms.size();
      DevTerm d{};
      d.coef = 1.0;
      d.K = (int32_t)cut.d[s];
      if (dir > 0) {
        d.a_buf = 0; d.a_off = goff[s]; d.lda = (int32_t)gn[s];
        d.b_buf = 1; d.b_off = goff[s]; d.ldb = (int32_t)gn[s];
      } else {
        d.a_buf = 1; d.a_off = goff[s]; d.lda = (int32_t)gn[s]; d.ops = 1 | 2;
        d.b_buf = 0; d.b_off = goff[s]; d.ldb = (int32_t)gn[s]; d.ops |= 4 | 8;
      }
      px.terms.push_back(d);
      ob.t_end = ob.d_begin = ob.d_end = (int32_t)px.terms.size();
      px.outs.push_back(ob);
    }
    b.p[0] = R2;
    b.p[1] = R1;
    if ((rc = run_program(ctx, px, b, (double*)x.data))) return rc;
    TDVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return TDVP_OK;
  }
  if (rc != TDVP_E_NOCONV) return rc;
  // Householder QR per sector (rank-deficient centre).  A failed round stops
  // before writing its output, so T still holds the original tensor.
  std::vector<int64_t> rows(ns, 0), moff(ns, 0), roff(T.n(), 0);
  for (int o = 0; o < T.n(); ++o) {
    const int sct = cut_sector(T, o, dir);
    roff[o] = rows[sct];
    rows[sct] += dir > 0 ? T.rows[o] : T.cols[o];
  }
  int64_t mtot = 0, ktot = 0;
  for (int sct = 0; sct < ns; ++sct) {
    if (rows[sct] < cut.d[sct])
      return set_error(ctx, TDVP_E_SHAPE, "one-site gauge move: bond larger than its support");
    moff[sct] = mtot;
    mtot += rows[sct] * cut.d[sct];
    ktot += cut.d[sct];
  }
  TDVP_HIP(ctx, ctx->ws_scratch.ensure(sizeof(double) * 2 * (size_t)(mtot + ktot + 1)));
  double* Mb = (double*)ctx->ws_scratch.p;
  double* tau = Mb + 2 * mtot;
  // gather M_s: dir +1 the (a, s) x d_b stack of the blocks; dir -1 the stack
  // of their conjugate transposes (the LQ of the row is a QR of its adjoint)
  Program pgat;
  for (int o = 0; o < T.n(); ++o) {
    const int sct = cut_sector(T, o, dir);
    DevOut ob{};
    ob.c_off = moff[sct] + roff[o];
    ob.ldc = (int32_t)rows[sct];
    ob.M = (int32_t)(dir > 0 ? T.rows[o] : T.cols[o]);
    ob.N = (int32_t)(dir > 0 ? T.cols[o] : T.rows[o]);
    ob.t_begin = ob.t_end = ob.d_begin = (int32_t)pgat.terms.size();
    DevTerm d{};
    d.a_buf = 0; d.a_off = T.off[o]; d.lda = (int32_t)T.rows[o];
    d.coef = 1.0;
    d.ops = dir > 0 ? 0 : (1 | 2);
    pgat.terms.push_back(d);
    ob.d_end = (int32_t)pgat.terms.size();
    pgat.outs.push_back(ob);
  }
  b.p[0] = (const double*)T.data;
  if ((rc = run_program(ctx, pgat, b, Mb))) return rc;
  // factor; keep R (upper d x d) in the R1 slots
  TDVP_HIP(ctx, hipMemsetAsync(R1, 0, sizeof(double) * 2 * (size_t)gtot, ctx->stream));
  int64_t kofs = 0;
  for (int sct = 0; sct < ns; ++sct) {
    const int64_t r = rows[sct], dd = cut.d[sct];
    auto* A = (rocblas_double_complex*)(Mb + 2 * moff[sct]);
    auto* tq = (rocblas_double_complex*)(tau + 2 * kofs);
    kofs += dd;
    rocblas_status st = rocsolver_zgeqrf((rocblas_handle)ctx->solver, (rocblas_int)r, (rocblas_int)dd, A,
                                         (rocblas_int)r, tq);
    if (st != rocblas_status_success) return set_error(ctx, TDVP_E_HIP, "rocsolver_zgeqrf failed");
    TDVP_HIP(ctx, hipMemcpy2DAsync(R1 + 2 * goff[sct], sizeof(double) * 2 * gn[sct], Mb + 2 * moff[sct],
                                   sizeof(double) * 2 * r, sizeof(double) * 2 * dd, dd, hipMemcpyDeviceToDevice,
                                   ctx->stream));
    st = rocsolver_zungqr((rocblas_handle)ctx->solver, (rocblas_int)r, (rocblas_int)dd, (rocblas_int)dd, A,
                          (rocblas_int)r, tq);
    if (st != rocblas_status_success) return set_error(ctx, TDVP_E_HIP, "rocsolver_zungqr failed");
  }
  for (auto& bk : buckets)
    if ((rc = vec_zero_lower(ctx, R1 + 2 * goff[bk.second.front()], bk.first, (int64_t)bk.second.size()))) return rc;
  // write back: the isometry into T, the triangle into x
  Program pw, px;
  for (int o = 0; o < T.n(); ++o) {
    const int sct = cut_sector(T, o, dir);
    DevOut ob{};
    ob.c_off = T.off[o];
    ob.ldc = ob.M = (int32_t)T.rows[o];
    ob.N = (int32_t)T.cols[o];
    ob.t_begin = ob.t_end = ob.d_begin = (int32_t)pw.terms.size();
    DevTerm d{};
    d.a_buf = 0; d.a_off = moff[sct] + roff[o]; d.lda = (int32_t)rows[sct];
    d.coef = 1.0;
    d.ops = dir > 0 ? 0 : (1 | 2);
    pw.terms.push_back(d);
    ob.d_end = (int32_t)pw.terms.size();
    pw.outs.push_back(ob);
  }
  for (int sct = 0; sct < ns; ++sct) {
    DevOut ob{};
    ob.c_off = x.off[sct];
    ob.ldc = ob.M = ob.N = (int32_t)cut.d[sct];
    ob.t_begin = ob.t_end = ob.d_begin = (int32_t)px.terms.size();
    DevTerm d{};
    d.a_buf = 1; d.a_off = goff[sct]; d.lda = (int32_t)gn[sct];
    d.coef = 1.0;
    d.ops = dir > 0 ? 0 : (1 | 2);
    px.terms.push_back(d);
    ob.d_end = (int32_t)px.terms.size();
    px.outs.push_back(ob);
  }
  b.p[0] = Mb;
  b.p[1] = R1;
  if ((rc = run_program(ctx, pw, b, (double*)T.data))) return rc;
  if ((rc = run_program(ctx, px, b, (double*)x.data))) return rc;
  TDVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (ctx->verbose) std::fprintf(stderr, "[tdvp]   site %d: Householder gauge move (dir %+d)\n", i, dir);
  return TDVP_OK;
}

}  // namespace
}  // namespace tdvp

namespace tdvp {
namespace {

// Backward evolution x <- exp(+i tau H0) x of the bond matrix after a gauge
// move at site i.  The zero-site effective Hamiltonian is the one-site one
// projected with the new isometry (the environment just built from it is
// exactly that projection): dir +1, x on bond i and H0 x = A^dag H1_i (A x);
// dir -1, x on bond i-1 and H0 x = (H1_i (x B)) B^dag.
int evolve_bond(tdvp_ctx* ctx, tdvp_mps* m, int i, int dir, Blocks& x, double tau_im, const tdvp_trunc& tr,
                tdvp_sweep_info* info) {
  const Blocks& T = m->site[i - 1]->blk;   // A_i (dir +1) or B_i (dir -1)
  HeffInputs in;
  in.sym = m->sym;
  in.l = m->bonds[i - 1];
  in.r = m->bonds[i];
  in.Le = m->Lenv[i - 1]->blk;
  in.Re = m->Renv[i]->blk;
  Blocks t1 = T;   // one-site layout of site i, compact scratch
  int rc;
  TDVP_HIP(ctx, ctx->ws_theta.ensure(sizeof(double) * 2 * (size_t)std::max<int64_t>(2 * T.size, 1)));
  double* t1d = (double*)ctx->ws_theta.p;
  double* t2d = t1d + 2 * T.size;
  t1.data = t1d;
  in.x = t1;
  Blocks t2 = T;
  t2.data = t2d;
  auto prog = heff_program(ctx, m->model, i, 1, in, t2, rc);
  if (rc) return rc;
  // pin: t1 = A x (dir +1) or x B (dir -1); pout: y = A^dag t2 or t2 B^dag
  Program pin, pout;
  double small_flops = 0.0;
  for (int o = 0; o < T.n(); ++o) {
    const int sct = cut_sector(T, o, dir);
    DevOut ob{};
    ob.c_off = T.off[o];
    ob.ldc = ob.M = (int32_t)T.rows[o];
    ob.N = (int32_t)T.cols[o];
    ob.t_begin = (int32_t)pin.terms.size();
    DevTerm d{};
    d.coef = 1.0;
    if (dir > 0) {
      d.a_buf = 0; d.a_off = T.off[o]; d.lda = (int32_t)T.rows[o];
      d.b_buf = 1; d.b_off = x.off[sct]; d.ldb = (int32_t)x.rows[sct];
      d.K = (int32_t)T.cols[o];
    } else {
      d.a_buf = 1; d.a_off = x.off[sct]; d.lda = (int32_t)x.rows[sct];
      d.b_buf = 0; d.b_off = T.off[o]; d.ldb = (int32_t)T.rows[o];
      d.K = (int32_t)T.rows[o];
    }
    small_flops += 8.0 * (double)T.rows[o] * (double)T.cols[o] * (double)d.K;
    pin.terms.push_back(d);
    ob.t_end = ob.d_begin = ob.d_end = (int32_t)pin.terms.size();
    pin.outs.push_back(ob);
  }
  for (int sct = 0; sct < x.n(); ++sct) {
    DevOut ob{};
    ob.c_off = x.off[sct];
    ob.ldc = ob.M = (int32_t)x.rows[sct];
    ob.N = (int32_t)x.cols[sct];
    ob.t_begin = (int32_t)pout.terms.size();
    for (int o = 0; o < T.n(); ++o) {
      if (cut_sector(T, o, dir) != sct) continue;
      DevTerm d{};
      d.coef = 1.0;
      if (dir > 0) {   // A^dag t2 over rows (a, s)
        d.a_buf = 0; d.a_off = T.off[o]; d.lda = (int32_t)T.rows[o]; d.ops = 1 | 2;
        d.b_buf = 2; d.b_off = T.off[o]; d.ldb = (int32_t)T.rows[o];
        d.K = (int32_t)T.rows[o];
      } else {         // t2 B^dag over columns (s, b)
        d.a_buf = 2; d.a_off = T.off[o]; d.lda = (int32_t)T.rows[o];
        d.b_buf = 0; d.b_off = T.off[o]; d.ldb = (int32_t)T.rows[o]; d.ops = 4 | 8;
        d.K = (int32_t)T.cols[o];
      }
      small_flops += 8.0 * (double)ob.M * (double)ob.N * (double)d.K;
      pout.terms.push_back(d);
    }
    ob.t_end = ob.d_begin = ob.d_end = (int32_t)pout.terms.size();
    pout.outs.push_back(ob);
  }
  pin.finalize();
  pout.finalize();
  if ((rc = upload(ctx, pin)) || (rc = upload(ctx, pout))) return rc;
  Bufs bh{};
  bh.p[0] = t1d;
  bh.p[1] = (const double*)in.Le.data;
  bh.p[2] = (const double*)in.Re.data;
  auto op = [&](const double* v, double* w) -> int {
    Bufs b{};
    b.p[0] = (const double*)T.data;
    b.p[1] = v;
    int r = launch_gemm(ctx, pin, b, t1d, ctx->precision);
    if (!r) r = launch_gemm(ctx, *prog, bh, t2d, ctx->precision);
    b.p[2] = t2d;
    if (!r) r = launch_gemm(ctx, pout, b, w, ctx->precision);
    return r;
  };
  KrylovResult kr;
  rc = krylov_core(ctx, x.size, (double*)x.data, op, prog->flops + small_flops, {0.0, tau_im}, tr.krylov_tol,
                   tr.krylov_maxdim, kr);
  info->krylov_iters += kr.iters;
  info->graph_iters += kr.graph_iters;
  info->krylov_max = std::max(info->krylov_max, kr.iters);
  info->heff_flops += kr.heff_flops;
  if (rc == TDVP_E_NOCONV) {
    info->nonconverged++;
    rc = TDVP_OK;
  }
  return rc;
}

// Move the bond matrix into the neighbour: dir +1, C_{i+1} = x B_{i+1};
// dir -1, C_{i-1} = A_{i-1} x.  Layouts are unchanged (same bond dimensions).
int absorb(tdvp_ctx* ctx, tdvp_mps* m, int i, int dir, const Blocks& x) {
  const int j = dir > 0 ? i + 1 : i - 1;   // receiving site
  Blocks& N = m->site[j - 1]->blk;
  TDVP_HIP(ctx, ctx->ws_theta.ensure(sizeof(double) * 2 * (size_t)std::max<int64_t>(N.size, 1)));
  double* tmp = (double*)ctx->ws_theta.p;
  Program p;
  for (int o = 0; o < N.n(); ++o) {
    const int sct = dir > 0 ? N.k(o)[0] : N.k(o)[2];
    DevOut ob{};
    ob.c_off = N.off[o];
    ob.ldc = ob.M = (int32_t)N.rows[o];
    ob.N = (int32_t)N.cols[o];
    ob.t_begin = (int32_t)p.terms.size();
    DevTerm d{};
    d.coef = 1.0;
    if (dir > 0) {
      d.a_buf = 1; d.a_off = x.off[sct]; d.lda = (int32_t)x.rows[sct];
      d.b_buf = 0; d.b_off = N.off[o]; d.ldb = (int32_t)N.rows[o];
      d.K = (int32_t)N.rows[o];
    } else {
      d.a_buf = 0; d.a_off = N.off[o]; d.lda = (int32_t)N.rows[o];
      d.b_buf = 1; d.b_off = x.off[sct]; d.ldb = (int32_t)x.rows[sct];
      d.K = (int32_t)N.cols[o];
    }
    p.terms.push_back(d);
    ob.t_end = ob.d_begin = ob.d_end = (int32_t)p.terms.size();
    p.outs.push_back(ob);
  }
  Bufs b{};
  b.p[0] = (const double*)N.data;
  b.p[1] = (const double*)x.data;
  int rc = run_program(ctx, p, b, tmp);
  if (rc) return rc;
  TDVP_HIP(ctx, hipMemcpyAsync(N.data, tmp, sizeof(double) * 2 * (size_t)N.size, hipMemcpyDeviceToDevice,
                               ctx->stream));
  return TDVP_OK;
}

}  // namespace
}  // namespace tdvp

// One time step dt of symmetric second-order one-site TDVP (bond dimensions fixed).
int tdvp_sweep1(tdvp_ctx* ctx, tdvp_mps* m, double dt, const tdvp_trunc* tr, tdvp_sweep_info* info) {
  if (!ctx || !m || !tr) return set_error(ctx, TDVP_E_INVALID, "null argument");
  return guarded(ctx, [&]() -> int {
    if (m->ctx != ctx) return set_error(ctx, TDVP_E_INVALID, "MPS belongs to another context");
    if (m->fragment) return set_error(ctx, TDVP_E_INVALID, "a split result is not a chain");
    if (tr->krylov_maxdim < 1 || tr->krylov_maxdim > 64) return set_error(ctx, TDVP_E_INVALID, "bad krylov_maxdim");
    TDVP_HIP(ctx, hipSetDevice(ctx->device));
    if (int r0 = unstage_all(ctx, m)) return r0;   // one-site sweeps keep every tensor on the device
    tdvp_sweep_info inf{};
    double t0 = now();
    const int L = m->L;
    const double tau = 0.5 * dt;
    int rc;
    Blocks x;
    DeviceBuffer xbuf, qbuf;
    use_alloc(ctx, {&xbuf, &qbuf});
    auto timed = [&](double& acc, auto&& f) -> int {
      double s = now();
      int r = f();
      acc += now() - s;
      return r;
    };
    auto site_evolve = [&](int i) {
      Blocks& c = m->site[i - 1]->blk;
      return timed(inf.t_lanczos, [&] {
        return evolve(ctx, m, i, 1, c, m->Lenv[i - 1]->blk, m->Renv[i]->blk, -tau, *tr, &inf);
      });
    };
    for (int i = 1; i <= L; ++i) {
      if ((rc = site_evolve(i))) return rc;
      if (i == L) break;
      if ((rc = timed(inf.t_svd, [&] { return gauge_qr(ctx, m, i, +1, x, xbuf, qbuf); }))) return rc;
      if ((rc = timed(inf.t_env, [&] { return env_step_sync(ctx, m, i, +1, &inf); }))) return rc;
      if ((rc = timed(inf.t_lanczos, [&] { return evolve_bond(ctx, m, i, +1, x, +tau, *tr, &inf); }))) return rc;
      if ((rc = absorb(ctx, m, i, +1, x))) return rc;
    }
    for (int i = L; i >= 1; --i) {
      if ((rc = site_evolve(i))) return rc;
      if (i == 1) break;
      if ((rc = timed(inf.t_svd, [&] { return gauge_qr(ctx, m, i, -1, x, xbuf, qbuf); }))) return rc;
      if ((rc = timed(inf.t_env, [&] { return env_step_sync(ctx, m, i, -1, &inf); }))) return rc;
      if ((rc = timed(inf.t_lanczos, [&] { return evolve_bond(ctx, m, i, -1, x, +tau, *tr, &inf); }))) return rc;
      if ((rc = absorb(ctx, m, i, -1, x))) return rc;
    }
    TDVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int k = 0; k <= L; ++k) {
      inf.max_chi = std::max(inf.max_chi, bond_chi(m->sym, m->bonds[k]));
      inf.max_chi_su2 = std::max(inf.max_chi_su2, m->bonds[k].chi_su2());
    }
    {
      bool bad = false;
      if ((rc = take_bad_flag(ctx, bad))) return rc;
      if (bad) return set_error(ctx, TDVP_E_NONFINITE, "non-finite values during the sweep");
    }
    inf.seconds = now() - t0;
    if (info) *info = inf;
    return TDVP_OK;
  });
}

// One time step of the adaptive scheme: two-site sweeps while the bond
// dimension grows, one-site sweeps once the largest bond has reached
// switch_frac of the cap (the mode is the caller's, so several runs can be
// kept on the same schedule).
int tdvp_step(tdvp_ctx* ctx, tdvp_mps* m, double dt, const tdvp_trunc* tr, double switch_frac, int32_t* mode,
              tdvp_sweep_info* info) {
  if (!ctx || !m || !tr || !mode) return set_error(ctx, TDVP_E_INVALID, "null argument");
  if (*mode != 0 && *mode != 1) return set_error(ctx, TDVP_E_INVALID, "mode must be 0 (two-site) or 1 (one-site)");
  if (std::isnan(switch_frac)) return set_error(ctx, TDVP_E_INVALID, "bad switch fraction");
  if (*mode == 1) return tdvp_sweep1(ctx, m, dt, tr, info);
  tdvp_sweep_info inf{};
  int rc = tdvp_sweep(ctx, m, dt, tr, &inf);
  if (info) *info = inf;
  if (rc) return rc;
  if (switch_frac > 0.0 && (double)inf.max_chi >= switch_frac * (double)tr->chi_cap) *mode = 1;
  return TDVP_OK;
}

// ---------------------------------------------------------------------------
// The two-site split as a call of its own (supplementary sections S2.2 and
// S2.4: per coupled sector of the bond, an SVD of the merged tensor, whole
// multiplets kept by discarded weight and bond-dimension cap).
namespace tdvp {
namespace {

// Coupled sectors x of the bond between the two sites, ascending (q, 2j),
// with the sizes of their sector matrices (rows: (a, s1), columns: (s2, b)).
void coupled_sectors(const Bond& l, const Bond& r, std::vector<std::array<int64_t, 4>>& out) {
  std::map<std::pair<int, int>, std::pair<int64_t, int64_t>> sec;
  for (int a = 0; a < l.size(); ++a)
    for (int s1 = 0; s1 < 3; ++s1)
      for (int tj = std::abs(l.tj[a] - kLocTJ[s1]); tj <= l.tj[a] + kLocTJ[s1]; tj += 2)
        sec[{l.q[a] + kLocQ[s1], tj}].first += l.d[a];
  for (auto& kv : sec)
    for (int s2 = 0; s2 < 3; ++s2)
      for (int b = 0; b < r.size(); ++b)
        if (kv.first.first + kLocQ[s2] == r.q[b] && triangle(kv.first.second, kLocTJ[s2], r.tj[b]))
          kv.second.second += r.d[b];
  out.clear();
  for (auto& kv : sec)
    if (kv.second.first > 0 && kv.second.second > 0)
      out.push_back({kv.first.first, kv.first.second, kv.second.first, kv.second.second});
}

}  // namespace
}  // namespace tdvp

extern "C" {

int tdvp_split_sectors(const tdvp_bond* left, const tdvp_bond* right, int32_t* nsec, int32_t* q, int32_t* tj,
                       int64_t* rows, int64_t* cols) {
  return guarded(nullptr, [&]() -> int {
    if (!left || !right || !nsec) return set_error(nullptr, TDVP_E_INVALID, "null argument");
    Bond l, r;
    std::string err;
    int rc = load_bond(l, left, err);
    if (!rc) rc = load_bond(r, right, err);
    if (rc) return set_error(nullptr, rc, err);
    std::vector<std::array<int64_t, 4>> sec;
    coupled_sectors(l, r, sec);
    *nsec = (int32_t)sec.size();
    for (size_t i = 0; i < sec.size(); ++i) {
      if (q) q[i] = (int32_t)sec[i][0];
      if (tj) tj[i] = (int32_t)sec[i][1];
      if (rows) rows[i] = sec[i][2];
      if (cols) cols[i] = sec[i][3];
    }
    return TDVP_OK;
  });
}

int tdvp_split(tdvp_ctx* ctx, const tdvp_bond* left, const tdvp_bond* right, const tdvp_blocks* theta,
               int32_t direction, const tdvp_trunc* trunc, tdvp_mps** out, double* svals, double* discarded) {
  if (!ctx) return set_error(nullptr, TDVP_E_INVALID, "null ctx");
  return guarded(ctx, [&]() -> int {
    if (!left || !right || !theta || !trunc || !out) return set_error(ctx, TDVP_E_INVALID, "null argument");
    *out = nullptr;
    if (direction != 1 && direction != -1) return set_error(ctx, TDVP_E_INVALID, "direction must be +1 or -1");
    if (!trunc->keep_all && !(trunc->eps_tol >= 0.0)) return set_error(ctx, TDVP_E_INVALID, "eps_tol must be >= 0");
    if (!trunc->keep_all && trunc->chi_cap < 1) return set_error(ctx, TDVP_E_INVALID, "chi_cap must be >= 1");
    TDVP_HIP(ctx, hipSetDevice(ctx->device));
    tdvp_model model{0.0, 0.0, 2};
    std::unique_ptr<tdvp_mps> m(new_mps(ctx, model));
    m->fragment = true;
    std::string err;
    int rc = load_bond(m->bonds[0], left, err);
    if (!rc) rc = load_bond(m->bonds[2], right, err);
    Blocks th;
    if (!rc) rc = load_center(th, theta, m->bonds[0], m->bonds[2], 2, err);
    if (rc) return set_error(ctx, rc, err);
    if (th.n() && !th.data) return set_error(ctx, TDVP_E_INVALID, "null device data pointer");
    // non-finite input is reported before the split
    if (th.size > 0) {
      TDVP_HIP(ctx, ctx->ws_small.ensure(1 << 16));
      double* d = (double*)ctx->ws_small.p + 1024;
      if ((rc = vec_norm2(ctx, (const double*)th.data, th.size, d))) return rc;
      double h[2];
      TDVP_HIP(ctx, hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
      TDVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
      if (h[1] != 0.0 || !std::isfinite(h[0])) return set_error(ctx, TDVP_E_NONFINITE, "non-finite entries in theta");
    }
    double disc = 0.0, t_svd = 0.0;
    int fallbacks = 0;
    std::vector<double> sv;
    if (th.size > 0 && (rc = split(ctx, m.get(), 1, th, direction, *trunc, disc, t_svd, fallbacks, &sv))) return rc;
    if (svals) std::copy(sv.begin(), sv.end(), svals);
    if (discarded) *discarded = disc;
    bool bad = false;
    if ((rc = take_bad_flag(ctx, bad))) return rc;
    if (bad) return set_error(ctx, TDVP_E_NONFINITE, "non-finite values in the split");
    *out = m.release();
    return TDVP_OK;
  });
}

}  // extern "C"

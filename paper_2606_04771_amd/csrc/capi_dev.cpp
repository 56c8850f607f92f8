// Device entry points of the C ABI: context, effective-Hamiltonian apply,
// Krylov exponential and environment update.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <cstdlib>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>

#include "common.hpp"
#include "ctx.hpp"
#include "device.hpp"
#include "tridiag.hpp"

using namespace tdvp;

namespace tdvp {

int hip_check(tdvp_ctx* ctx, hipError_t e, const char* what) {
  const int code = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? TDVP_E_NOMEM : TDVP_E_HIP;
  return set_error(ctx, code, std::string(what) + ": " + hipGetErrorString(e));
}

namespace {

// Structural hash of a program's inputs; the values hashed are also kept, so
// that a cache hit can be confirmed by comparing them.
struct Hasher {
  uint64_t h = 1469598103934665603ull;
  std::vector<uint64_t> sig;
  void add(uint64_t v) {
    sig.push_back(v);
    h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    h *= 1099511628211ull;
  }
  void addd(double d) {
    uint64_t v;
    std::memcpy(&v, &d, 8);
    add(v);
  }
  void blocks(const Blocks& b) {
    add((uint64_t)b.n());
    for (int v : b.key) add((uint64_t)(int64_t)v);
    for (auto v : b.off) add((uint64_t)v);
  }
  void bond(const Bond& b) {
    add((uint64_t)b.size());
    for (int i = 0; i < b.size(); ++i) {
      add((uint64_t)(int64_t)b.q[i]);
      add((uint64_t)b.tj[i]);
      add((uint64_t)b.d[i]);
    }
  }
};

}  // namespace

int take_bad_flag(tdvp_ctx* ctx, bool& bad) {
  bad = false;
  if (!ctx->ws_flag.p) return TDVP_OK;
  int h = 0;
  TDVP_HIP(ctx, hipMemcpyAsync(&h, ctx->ws_flag.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  TDVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (h) {
    TDVP_HIP(ctx, hipMemsetAsync(ctx->ws_flag.p, 0, sizeof(int), ctx->stream));
    TDVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    bad = true;
  }
  return TDVP_OK;
}

// Lower an H_eff plan to a grouped-GEMM program.  Buffers: 0 = x, 1 = Lenv,
// 2 = Renv; output blocks at y's offsets.
std::shared_ptr<Program> heff_program(tdvp_ctx* ctx, const tdvp_model& m, int site, int nsites,
                                      const HeffInputs& in, const Blocks& y, int& rc) {
  Hasher hs;
  hs.add(1);
  hs.addd(m.t);
  hs.addd(m.U);
  hs.add((uint64_t)site);
  hs.add((uint64_t)nsites);
  hs.bond(in.l);
  hs.bond(in.r);
  hs.blocks(in.Le);
  hs.blocks(in.Re);
  hs.blocks(in.x);
  hs.blocks(y);
  hs.addd(ctx->split_alpha);
  hs.add((uint64_t)ctx->split_kmin);
  hs.add((uint64_t)in.sym);
  rc = TDVP_OK;
  if (auto p = cache_get(ctx, hs.h, hs.sig)) return p;
  std::vector<HTerm> terms;
  double flops = 0;
  if (in.sym == 1) u1_plan_heff(m, site, nsites, in.l, in.r, in.Le, in.Re, in.x, terms, flops);
  else plan_heff(m, site, nsites, in.l, in.r, in.Le, in.Re, in.x, terms, flops);
  std::stable_sort(terms.begin(), terms.end(), [](const HTerm& a, const HTerm& b) { return a.out < b.out; });
  auto p = std::make_shared<Program>();
  p->flops = flops;
  p->role = 1;
  p->sig = hs.sig;
  p->split_alpha = ctx->split_alpha;
  p->split_kmin = ctx->split_kmin;
  size_t t = 0;
  const Blocks& x = in.x;
  std::vector<DevTerm> direct;
  for (int o = 0; o < x.n(); ++o) {
    DevOut ob{};
    ob.c_off = y.off[o];
    ob.ldc = (int32_t)x.rows[o];
    ob.M = (int32_t)x.rows[o];
    ob.N = (int32_t)x.cols[o];
    ob.t_begin = (int32_t)p->terms.size();
    direct.clear();
    for (; t < terms.size() && terms[t].out == o; ++t) {
      const HTerm& h = terms[t];
      DevTerm d{};
      d.coef = h.coef;
      // block-Hamiltonian terms (channel H, diagonal in the sector) carry the
      // diagonal shift of their environment, compensated by a direct term
      auto shifted = [&](const Blocks& E, int bit) {
        if (E.k(h.env)[1] != 0 || h.in != h.out) return;
        d.ops |= bit;
        DevTerm c{};
        c.a_buf = 0; c.a_off = x.off[h.in]; c.lda = (int32_t)x.rows[h.in];
        c.K = 0; c.coef = h.coef; c.ops = bit;
        direct.push_back(c);
      };
      if (h.kind == 0) {   // E(a', a) . x(a, .)
        d.a_buf = 1; d.a_off = in.Le.off[h.env]; d.lda = (int32_t)in.Le.rows[h.env];
        d.b_buf = 0; d.b_off = x.off[h.in]; d.ldb = (int32_t)x.rows[h.in];
        d.K = (int32_t)x.rows[h.in];
        d.ops = 0;
        shifted(in.Le, 16);
        p->terms.push_back(d);
      } else if (h.kind == 1) {   // x(., b) . E(b', b)^T
        d.a_buf = 0; d.a_off = x.off[h.in]; d.lda = (int32_t)x.rows[h.in];
        d.b_buf = 2; d.b_off = in.Re.off[h.env]; d.ldb = (int32_t)in.Re.rows[h.env];
        d.K = (int32_t)x.cols[h.in];
        d.ops = 4;
        shifted(in.Re, 32);
        p->terms.push_back(d);
      } else {
        d.a_buf = 0; d.a_off = x.off[h.in]; d.lda = (int32_t)x.rows[h.in];
        d.K = 0;
        direct.push_back(d);
      }
    }
    ob.t_end = (int32_t)p->terms.size();
    ob.d_begin = (int32_t)p->terms.size();
    p->terms.insert(p->terms.end(), direct.begin(), direct.end());
    ob.d_end = (int32_t)p->terms.size();
    p->outs.push_back(ob);
  }
  // diagonal blocks of the block-Hamiltonian channels (shifts of reduced-precision launches)
  const Blocks* E[2] = {&in.Le, &in.Re};
  const Bond* B[2] = {&in.l, &in.r};
  for (int s = 0; s < 2; ++s)
    for (int i = 0; i < E[s]->n(); ++i) {
      const int* k = E[s]->k(i);
      if (k[1] != 0 || k[0] != k[2] || E[s]->rows[i] != E[s]->cols[i]) continue;
      p->shift_meta.push_back(E[s]->off[i]);
      p->shift_meta.push_back(E[s]->rows[i]);
      p->shift_meta.push_back(in.sym == 1 ? 1 : B[s]->tj[k[0]] + 1);   // multiplet weight
      p->nshift[s]++;
    }
  p->finalize();
  rc = upload(ctx, *p);
  if (rc) return nullptr;
  cache_put(ctx, hs.h, p);
  return p;
}

// Environment update as two grouped-GEMM programs: stage 1 writes the
// products E . op(ket) into scratch (buffer 3), stage 2 contracts them (or the
// ket directly) with op(bra)^ into the output environment.
// Buffers: 1 = env_in, 2 = tensor, 3 = scratch.
namespace {

Hasher env_hash(tdvp_ctx* ctx, const tdvp_model& m, int site, int dir, const EnvInputs& in) {
  Hasher hs;
  hs.add(2);
  hs.addd(m.t);
  hs.addd(m.U);
  hs.add((uint64_t)site);
  hs.add((uint64_t)(dir + 2));
  hs.bond(in.bin);
  hs.bond(in.bout);
  hs.blocks(in.ein);
  hs.blocks(in.ten);
  hs.blocks(in.eout);
  hs.addd(ctx->split_alpha);
  hs.add((uint64_t)ctx->split_kmin);
  hs.add((uint64_t)in.sym);
  return hs;
}

constexpr uint64_t kStage2Key = 0x5555555555555555ull;

// Host side of the two stages (term lists, tiles); nothing on the device.
EnvPrograms build_env_programs(tdvp_ctx* ctx, const tdvp_model& m, int site, int dir, const EnvInputs& in,
                               const Hasher& hs) {
  std::vector<ETerm> terms;
  double flops = 0;
  if (in.sym == 1) u1_plan_env(m, site, dir, in.bin, in.bout, in.ein, in.ten, in.eout, terms, flops);
  else plan_env(m, site, dir, in.bin, in.bout, in.ein, in.ten, in.eout, terms, flops);
  std::stable_sort(terms.begin(), terms.end(), [](const ETerm& a, const ETerm& b) { return a.out < b.out; });
  const Blocks &E = in.ein, &T = in.ten, &O = in.eout;
  // stage 1: one output per distinct (env, ket) pair
  auto s1 = std::make_shared<Program>();
  std::map<std::pair<int, int>, std::pair<int64_t, int>> prod;   // -> (scratch offset, rows)
  int64_t so = 0;
  for (const ETerm& e : terms) {
    if (e.kind != 0) continue;
    auto key = std::make_pair(e.env, e.ket);
    if (prod.count(key)) continue;
    int64_t rows = E.rows[e.env];
    int64_t cols = dir > 0 ? T.cols[e.ket] : T.rows[e.ket];
    prod[key] = {so, (int)rows};
    DevOut ob{};
    ob.c_off = so;
    ob.ldc = (int32_t)rows;
    ob.M = (int32_t)rows;
    ob.N = (int32_t)cols;
    ob.t_begin = (int32_t)s1->terms.size();
    DevTerm d{};
    d.coef = 1.0;
    d.a_buf = 1; d.a_off = E.off[e.env]; d.lda = (int32_t)E.rows[e.env];
    d.b_buf = 2; d.b_off = T.off[e.ket]; d.ldb = (int32_t)T.rows[e.ket];
    d.K = (int32_t)E.cols[e.env];
    d.ops = dir > 0 ? 0 : 4;
    s1->terms.push_back(d);
    ob.t_end = ob.d_begin = ob.d_end = (int32_t)s1->terms.size();
    s1->outs.push_back(ob);
    so += rows * cols;
  }
  s1->aux = so;
  s1->sig = hs.sig;
  if (ctx->split_alpha >= 0.0) {   // an explicit setting applies to the environment stages too
    s1->split_alpha = ctx->split_alpha;
    s1->split_kmin = ctx->split_kmin;
  }
  s1->finalize();
  // stage 2
  auto s2 = std::make_shared<Program>();
  s2->flops = flops;
  s2->sig = hs.sig;
  if (ctx->split_alpha >= 0.0) {
    s2->split_alpha = ctx->split_alpha;
    s2->split_kmin = ctx->split_kmin;
  }
  size_t t = 0;
  for (int o = 0; o < O.n(); ++o) {
    DevOut ob{};
    ob.c_off = O.off[o];
    ob.ldc = (int32_t)O.rows[o];
    ob.M = (int32_t)O.rows[o];
    ob.N = (int32_t)O.cols[o];
    ob.t_begin = (int32_t)s2->terms.size();
    for (; t < terms.size() && terms[t].out == o; ++t) {
      const ETerm& e = terms[t];
      DevTerm d{};
      d.coef = e.coef;
      d.a_buf = 2; d.a_off = T.off[e.bra]; d.lda = (int32_t)T.rows[e.bra];
      d.ops = dir > 0 ? 3 : 2;           // A^dag (left) or conj(B) (right)
      if (e.kind == 0) {
        auto pr = prod.at({e.env, e.ket});
        d.b_buf = 3; d.b_off = pr.first; d.ldb = pr.second;
      } else {
        d.b_buf = 2; d.b_off = T.off[e.ket]; d.ldb = (int32_t)T.rows[e.ket];
        d.ops |= dir > 0 ? 0 : 4;       // A (left) or B^T (right)
      }
      d.K = (int32_t)(dir > 0 ? T.rows[e.bra] : T.cols[e.bra]);
      s2->terms.push_back(d);
    }
    ob.t_end = ob.d_begin = ob.d_end = (int32_t)s2->terms.size();
    s2->outs.push_back(ob);
  }
  s2->finalize();
  EnvPrograms ep;
  ep.s1 = s1;
  ep.s2 = s2;
  ep.scratch = so;
  return ep;
}

}  // namespace

EnvPrograms env_programs(tdvp_ctx* ctx, const tdvp_model& m, int site, int dir, const EnvInputs& in, int& rc) {
  const Hasher hs = env_hash(ctx, m, site, dir, in);
  rc = TDVP_OK;
  EnvPrograms ep;
  auto p1 = cache_get(ctx, hs.h, hs.sig);
  auto p2 = cache_get(ctx, hs.h ^ kStage2Key, hs.sig);
  if (p1 && p2) {
    ep.s1 = p1;
    ep.s2 = p2;
    ep.scratch = p1->aux;
    return ep;
  }
  ep = build_env_programs(ctx, m, site, dir, in, hs);
  rc = upload(ctx, *ep.s1);
  if (!rc) rc = upload(ctx, *ep.s2);
  if (rc) return EnvPrograms{};
  cache_put(ctx, hs.h, ep.s1);
  cache_put(ctx, hs.h ^ kStage2Key, ep.s2);
  return ep;
}

EnvPrograms env_programs_host(tdvp_ctx* ctx, const tdvp_model& m, int site, int dir, const EnvInputs& in) {
  const Hasher hs = env_hash(ctx, m, site, dir, in);
  EnvPrograms ep;
  // the device cache holds the same host description of uploaded programs
  auto p1 = cache_get(ctx, hs.h, hs.sig);
  auto p2 = cache_get(ctx, hs.h ^ kStage2Key, hs.sig);
  if (!(p1 && p2)) {
    p1 = cache_get(ctx->host_cache, hs.h, hs.sig);
    p2 = cache_get(ctx->host_cache, hs.h ^ kStage2Key, hs.sig);
  }
  if (p1 && p2) {
    ep.s1 = p1;
    ep.s2 = p2;
    ep.scratch = p1->aux;
    return ep;
  }
  ep = build_env_programs(ctx, m, site, dir, in, hs);
  cache_put(ctx->host_cache, hs.h, ep.s1);
  cache_put(ctx->host_cache, hs.h ^ kStage2Key, ep.s2);
  return ep;
}

int env_update_dev(tdvp_ctx* ctx, const tdvp_model& m, int site, int dir, const EnvInputs& in, double* flops) {
  int rc;
  EnvPrograms ep = env_programs(ctx, m, site, dir, in, rc);
  if (rc) return rc;
  if (flops) *flops = ep.s2->flops;
  TDVP_HIP(ctx, ctx->ws_scratch.ensure(sizeof(double) * 2 * (size_t)std::max<int64_t>(ep.scratch, 1)));
  Bufs b{};
  b.p[1] = (const double*)in.ein.data;
  b.p[2] = (const double*)in.ten.data;
  b.p[3] = (const double*)ctx->ws_scratch.p;
  rc = launch_gemm(ctx, *ep.s1, b, (double*)ctx->ws_scratch.p, ctx->precision);
  if (rc) return rc;
  return launch_gemm(ctx, *ep.s2, b, (double*)in.eout.data, ctx->precision);
}

}  // namespace tdvp

extern "C" {

int tdvp_ctx_create(tdvp_ctx** out, int32_t device, void* hip_stream, int32_t precision,
                    void* (*dev_alloc)(size_t, void*), void (*dev_free)(void*, void*), void* user) {
  return guarded(nullptr, [&]() -> int {
    if ((dev_alloc == nullptr) != (dev_free == nullptr))
      return set_error(nullptr, TDVP_E_INVALID, "dev_alloc and dev_free must be given together");
    if (!out) return set_error(nullptr, TDVP_E_INVALID, "out is null");
    *out = nullptr;
    if (precision != TDVP_FP64 && precision != TDVP_FP32 && precision != TDVP_BF16X3)
      return set_error(nullptr, TDVP_E_INVALID, "unknown precision");
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) return set_error(nullptr, TDVP_E_HIP, "no HIP device available");
    if (device < 0 || device >= n) return set_error(nullptr, TDVP_E_INVALID, "bad device ordinal");
    e = hipSetDevice(device);
    if (e != hipSuccess) return set_error(nullptr, TDVP_E_HIP, hipGetErrorString(e));
    auto* c = new tdvp_ctx();
    c->device = device;
    c->precision = precision;
    {
      auto al = std::make_shared<Allocator>();
      al->alloc_fn = dev_alloc;
      al->free_fn = dev_free;
      al->user = user;
      c->alloc = al;
      c->pool->al = al;
      for (DeviceBuffer* b : {&c->ws_scratch, &c->ws_krylov, &c->ws_small, &c->ws_vec, &c->ws_theta, &c->ws_svd,
                              &c->ws_lanczos, &c->ws_part, &c->ws_shift, &c->ws_compact, &c->ws_flag, &c->ws_slices,
                              &c->ws_trd})
        b->al = al;
    }
    if (const char* e = std::getenv("TDVP_SPLIT_ALPHA")) c->split_alpha = std::atof(e);
    if (const char* e = std::getenv("TDVP_SPLIT_KMIN")) c->split_kmin = std::max(1, std::atoi(e));
    if (hip_stream) {
      c->stream = (hipStream_t)hip_stream;
    } else {
      e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
      if (e != hipSuccess) {
        delete c;
        return set_error(nullptr, TDVP_E_HIP, hipGetErrorString(e));
      }
      c->own_stream = true;
    }
    e = hipHostMalloc(&c->host_small, 1 << 16);
    if (e != hipSuccess) {
      delete c;
      return set_error(nullptr, TDVP_E_NOMEM, "pinned host buffer");
    }
    // the non-finite flag, zeroed before any launch can be recorded into a graph
    e = c->ws_flag.ensure(256);
    if (e == hipSuccess) e = hipMemsetAsync(c->ws_flag.p, 0, 256, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
      if (c->own_stream) (void)hipStreamDestroy(c->stream);
      if (c->host_small) (void)hipHostFree(c->host_small);
      delete c;
      return set_error(nullptr, e == hipErrorOutOfMemory ? TDVP_E_NOMEM : TDVP_E_HIP, "context flag buffer");
    }
    for (auto& ev : c->ev) (void)hipEventCreate(&ev);
    // device address of the static scratch of the allocation-free entry point
    // (once per device, with the device current) and the event that orders
    // reuse of its host staging
    if (int rc = noalloc_init(c)) {
      std::string msg = c->err;
      for (auto& ev : c->ev)
        if (ev) (void)hipEventDestroy(ev);
      if (c->own_stream) (void)hipStreamDestroy(c->stream);
      if (c->host_small) (void)hipHostFree(c->host_small);
      delete c;
      return set_error(nullptr, rc, msg);
    }
    (void)hipEventCreateWithFlags(&c->na_copied, hipEventDisableTiming);
    const char* gr = std::getenv("TDVP_GRAPH");
    c->graphs = !(gr && std::atoi(gr) == 0);
    const char* v = std::getenv("TDVP_VERBOSE");
    c->verbose = v ? std::atoi(v) : 0;
    *out = c;
    return TDVP_OK;
  });
}

void tdvp_ctx_destroy(tdvp_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  ctx->cache.clear();
  if (ctx->solver) (void)rocblas_destroy_handle((rocblas_handle)ctx->solver);
  for (int k = 0; k < tdvp_ctx::kSide; ++k) {
    if (ctx->side[k]) (void)hipStreamSynchronize(ctx->side[k]);
    if (ctx->side_solver[k]) (void)rocblas_destroy_handle((rocblas_handle)ctx->side_solver[k]);
    if (ctx->side[k]) (void)hipStreamDestroy(ctx->side[k]);
  }
  for (auto& ev : ctx->side_ev)
    if (ev) (void)hipEventDestroy(ev);
  for (auto& ev : ctx->eig_ev) (void)hipEventDestroy(ev);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->host_small) (void)hipHostFree(ctx->host_small);
  if (ctx->upload_done) (void)hipEventDestroy(ctx->upload_done);
  if (ctx->na_copied) (void)hipEventDestroy(ctx->na_copied);
  for (auto& ev : ctx->ev)
    if (ev) (void)hipEventDestroy(ev);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

int tdvp_ctx_set_precision(tdvp_ctx* ctx, int32_t precision) {
  if (!ctx) return set_error(nullptr, TDVP_E_INVALID, "null ctx");
  if (precision != TDVP_FP64 && precision != TDVP_FP32 && precision != TDVP_BF16X3)
    return set_error(ctx, TDVP_E_INVALID, "unknown precision");
  ctx->precision = precision;
  return TDVP_OK;
}

int tdvp_ctx_set_krylov_storage(tdvp_ctx* ctx, int32_t precision) {
  if (!ctx) return set_error(nullptr, TDVP_E_INVALID, "null ctx");
  if (precision != TDVP_FP64 && precision != TDVP_FP32)
    return set_error(ctx, TDVP_E_INVALID, "Krylov basis storage must be TDVP_FP64 or TDVP_FP32");
  ctx->krylov_fp32 = precision == TDVP_FP32;
  return TDVP_OK;
}

int tdvp_ctx_set_host_staging(tdvp_ctx* ctx, int32_t enable) {
  if (!ctx) return set_error(nullptr, TDVP_E_INVALID, "null ctx");
  ctx->host_staging = enable != 0;
  return TDVP_OK;
}

int tdvp_ctx_memory(tdvp_ctx* ctx, int64_t* live_bytes, int64_t* peak_bytes, int32_t reset_peak) {
  if (!ctx) return set_error(nullptr, TDVP_E_INVALID, "null ctx");
  std::lock_guard<std::mutex> lk(ctx->alloc->mu);
  if (live_bytes) *live_bytes = (int64_t)ctx->alloc->live;
  if (peak_bytes) *peak_bytes = (int64_t)ctx->alloc->peak;
  if (reset_peak) ctx->alloc->peak = ctx->alloc->live;
  return TDVP_OK;
}

int tdvp_ctx_set_graphs(tdvp_ctx* ctx, int32_t enable) {
  if (!ctx) return set_error(nullptr, TDVP_E_INVALID, "null ctx");
  ctx->graphs = enable != 0;
  return TDVP_OK;
}

int tdvp_ctx_set_split(tdvp_ctx* ctx, double alpha, int32_t kmin) {
  if (!ctx) return set_error(nullptr, TDVP_E_INVALID, "null ctx");
  if (std::isnan(alpha) || kmin < 1) return set_error(ctx, TDVP_E_INVALID, "bad split parameters");
  ctx->split_alpha = alpha < 0.0 ? -1.0 : alpha;
  ctx->split_kmin = kmin;
  return TDVP_OK;
}

int tdvp_ctx_synchronize(tdvp_ctx* ctx) {
  if (!ctx) return set_error(nullptr, TDVP_E_INVALID, "null ctx");
  TDVP_HIP(ctx, hipSetDevice(ctx->device));
  TDVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  bool bad = false;
  if (int rc = take_bad_flag(ctx, bad)) return rc;
  if (bad) return set_error(ctx, TDVP_E_NONFINITE, "an earlier apply or environment update produced non-finite values");
  return TDVP_OK;
}

const char* tdvp_last_error(const tdvp_ctx* ctx) { return get_error(ctx); }

int tdvp_tridiag_expm(int32_t n, const double* alpha, const double* beta, double tau_re, double tau_im,
                      double nrm, double* y) {
  return guarded(nullptr, [&]() -> int {
    if (n < 1 || !alpha || (n > 1 && !beta) || !y) return set_error(nullptr, TDVP_E_INVALID, "bad arguments");
    std::vector<double> a(alpha, alpha + n), b(n > 1 ? beta : alpha, n > 1 ? beta + n - 1 : alpha);
    std::vector<std::complex<double>> out;
    if (!tridiag_expm_e1(a, b, {tau_re, tau_im}, nrm, out))
      return set_error(nullptr, TDVP_E_NOCONV, "tridiagonal eigensolver did not converge");
    for (int i = 0; i < n; ++i) {
      y[2 * i] = out[i].real();
      y[2 * i + 1] = out[i].imag();
    }
    return TDVP_OK;
  });
}

int tdvp_heff_apply(tdvp_ctx* ctx, const tdvp_model* model, int32_t site, int32_t nsites, const tdvp_bond* left,
                    const tdvp_bond* right, const tdvp_blocks* Lenv, const tdvp_blocks* Renv, const tdvp_blocks* x,
                    tdvp_blocks* y) {
  if (!ctx) return set_error(nullptr, TDVP_E_INVALID, "null ctx");
  return guarded(ctx, [&]() -> int {
    HeffInputs in;
    std::string err;
    int rc = load_heff_inputs(in, model, site, nsites, left, right, Lenv, Renv, x, err);
    Blocks yb;
    if (!rc) rc = match_keys(in.x, yb, y, err);
    if (rc) return set_error(ctx, rc, err);
    if ((in.x.n() && (!in.x.data || !yb.data)) || (in.Le.n() && !in.Le.data) || (in.Re.n() && !in.Re.data))
      return set_error(ctx, TDVP_E_INVALID, "null device data pointer");
    TDVP_HIP(ctx, hipSetDevice(ctx->device));
    auto p = heff_program(ctx, *model, site, nsites, in, yb, rc);
    if (rc) return rc;
    Bufs b{};
    b.p[0] = (const double*)in.x.data;
    b.p[1] = (const double*)in.Le.data;
    b.p[2] = (const double*)in.Re.data;
    return launch_gemm(ctx, *p, b, (double*)yb.data, ctx->precision);
  });
}

int tdvp_env_update(tdvp_ctx* ctx, const tdvp_model* model, int32_t site, int32_t direction,
                    const tdvp_bond* bond_in, const tdvp_bond* bond_out, const tdvp_blocks* env_in,
                    const tdvp_blocks* tensor, tdvp_blocks* env_out) {
  if (!ctx) return set_error(nullptr, TDVP_E_INVALID, "null ctx");
  return guarded(ctx, [&]() -> int {
    EnvInputs in;
    std::string err;
    int rc = load_env_inputs(in, model, site, direction, bond_in, bond_out, env_in, tensor, env_out, err);
    if (rc) return set_error(ctx, rc, err);
    if ((in.ten.n() && !in.ten.data) || (in.eout.n() && !in.eout.data) || (in.ein.n() && !in.ein.data))
      return set_error(ctx, TDVP_E_INVALID, "null device data pointer");
    TDVP_HIP(ctx, hipSetDevice(ctx->device));
    return env_update_dev(ctx, *model, site, direction, in);
  });
}

int tdvp_krylov_expm(tdvp_ctx* ctx, const tdvp_model* model, int32_t site, int32_t nsites, const tdvp_bond* left,
                     const tdvp_bond* right, const tdvp_blocks* Lenv, const tdvp_blocks* Renv, tdvp_blocks* x,
                     double tau_re, double tau_im, double tol, int32_t maxdim, tdvp_krylov_info* info) {
  if (!ctx) return set_error(nullptr, TDVP_E_INVALID, "null ctx");
  return guarded(ctx, [&]() -> int {
    HeffInputs in;
    std::string err;
    int rc = load_heff_inputs(in, model, site, nsites, left, right, Lenv, Renv, x, err);
    if (rc) return set_error(ctx, rc, err);
    if (maxdim < 1 || maxdim > 64) return set_error(ctx, TDVP_E_INVALID, "maxdim must be in 1..64");
    if (!(tol >= 0.0)) return set_error(ctx, TDVP_E_INVALID, "tol must be >= 0");
    TDVP_HIP(ctx, hipSetDevice(ctx->device));
    KrylovResult kr;
    rc = krylov_dev(ctx, *model, site, nsites, in, {tau_re, tau_im}, tol, maxdim, kr);
    if (rc == TDVP_OK || rc == TDVP_E_NOCONV || rc == TDVP_E_NONFINITE) {
      bool bad = false;
      if (int r2 = take_bad_flag(ctx, bad)) return r2;
      if (bad && rc != TDVP_E_NONFINITE) rc = set_error(ctx, TDVP_E_NONFINITE, "non-finite values in the Krylov exponential");
    }
    if (info) {
      std::memset(info, 0, sizeof(*info));
      info->iters = kr.iters;
      info->graph_iters = kr.graph_iters;
      info->converged = kr.converged;
      info->err_est = kr.err;
      info->norm_in = kr.norm;
      for (int i = 0; i < kr.iters && i < 64; ++i) info->alpha[i] = kr.alpha[i];
      for (int i = 0; i < kr.iters && i < 64 && i < (int)kr.beta.size(); ++i) info->beta[i] = kr.beta[i];
    }
    return rc;
  });
}

}  // extern "C"

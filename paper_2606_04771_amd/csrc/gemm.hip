// Output-stationary grouped complex GEMM on CDNA4 matrix cores.
//
// One launch evaluates every output block of an effective-Hamiltonian apply
// (or an environment-update stage): each output tile sums all of its
// contributing block products (left-environment, right-environment and
// local terms, each with its recoupling coefficient) in registers and is
// written once.  No atomics, a fixed summation order, so results are
// bit-reproducible.  The paper batches equal-size blocks into batched GEMMs
// (supplementary section S2.3); here uneven blocks go out in one grid whose
// tiles are ordered by decreasing work, so the hardware dispatcher hands the
// longest tiles out first.
//
// Tiles are 64x64 (four waves, each owning 32x32) by default; 32x32 tiles with
// one wave are selectable.  Measured at chi = 4096 the 64x64 tiling is the
// faster one despite more padding (57 % of issued matrix work useful against
// 76 %): it halves the operand traffic per flop.
// FP64 path: v_mfma_f64_16x16x4_f64, complex products as four real products
// on planar (re, im) LDS tiles.  Lane layout of the instruction: A[i][k] in
// lane i + 16 k, B[k][j] in lane j + 16 k, D[4 r + l/16][l % 16] in register r.
// FP32 path: the same tiling on v_mfma_f32_16x16x4_f32 with FP32 operands and
// accumulators (D[4 (l/16) + r][l % 16]), converted from and to FP64 at the
// tile boundary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "ctx.hpp"

namespace tdvp {

namespace {

constexpr int TK = 16, PAD = 2;

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// MFMA flavours: FP64 16x16x4 writes D[4 r + l/16][l%16], FP32 16x16x4 writes D[4 (l/16) + r][l%16].
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef f64x4 acc_t;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int r, int lk) { return 4 * r + lk; }
};
template <> struct Mfma<float> {
  typedef f32x4 acc_t;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int r, int lk) { return 4 * lk + r; }
};

// Tile TM x TN = (32 WM) x (32 WN); WM x WN waves, each owning a 32x32 sub-tile.
template <int WM, int WN>
struct Shape {
  static constexpr int TM = 32 * WM, TN = 32 * WN, NT = 64 * WM * WN;
  static constexpr int NA = TM * TK / NT, NB = TK * TN / NT;   // elements per thread
};

template <int WM, int WN>
struct Stage {
  double2 a[Shape<WM, WN>::NA], b[Shape<WM, WN>::NB];
};

// Load this thread's A and B elements of the K-tile k0 of term tm (coalesced:
// consecutive threads follow the contiguous dimension of each operand).
template <int WM, int WN>
__device__ __forceinline__ void load_stage(Stage<WM, WN>& st, const DevTerm& tm, const Bufs& bufs, int m0, int n0,
                                           int M, int N, int k0, int tid) {
  typedef Shape<WM, WN> S;
  const double2* A = reinterpret_cast<const double2*>(bufs.p[tm.a_buf]) + tm.a_off;
  const double2* B = reinterpret_cast<const double2*>(bufs.p[tm.b_buf]) + tm.b_off;
  const bool ta = tm.ops & 1, tb = tm.ops & 4;
#pragma unroll
  for (int r = 0; r < S::NA; ++r) {
    int e = tid + S::NT * r;
    int m = ta ? (e / TK) : (e % S::TM);
    int k = ta ? (e % TK) : (e / S::TM);
    int gm = m0 + m, gk = k0 + k;
    double2 v = make_double2(0.0, 0.0);
    if (gm < M && gk < tm.K)
      v = ta ? A[(int64_t)gk + (int64_t)gm * tm.lda] : A[(int64_t)gm + (int64_t)gk * tm.lda];
    st.a[r] = v;
  }
#pragma unroll
  for (int r = 0; r < S::NB; ++r) {
    int e = tid + S::NT * r;
    int n = tb ? (e % S::TN) : (e / TK);
    int k = tb ? (e / S::TN) : (e % TK);
    int gn = n0 + n, gk = k0 + k;
    double2 v = make_double2(0.0, 0.0);
    if (gn < N && gk < tm.K)
      v = tb ? B[(int64_t)gn + (int64_t)gk * tm.ldb] : B[(int64_t)gk + (int64_t)gn * tm.ldb];
    st.b[r] = v;
  }
}

template <typename T, int WM, int WN>
__device__ __forceinline__ void store_stage(const Stage<WM, WN>& st, const DevTerm& tm,
                                            T (*As)[TK][Shape<WM, WN>::TM + PAD],
                                            T (*Bs)[TK][Shape<WM, WN>::TN + PAD], int tid) {
  typedef Shape<WM, WN> S;
  const bool ta = tm.ops & 1, ca = tm.ops & 2, tb = tm.ops & 4, cb = tm.ops & 8;
  const double c = tm.coef;
#pragma unroll
  for (int r = 0; r < S::NA; ++r) {
    int e = tid + S::NT * r;
    int m = ta ? (e / TK) : (e % S::TM);
    int k = ta ? (e % TK) : (e / S::TM);
    As[0][k][m] = (T)(c * st.a[r].x);
    As[1][k][m] = (T)(ca ? -c * st.a[r].y : c * st.a[r].y);
  }
#pragma unroll
  for (int r = 0; r < S::NB; ++r) {
    int e = tid + S::NT * r;
    int n = tb ? (e % S::TN) : (e / TK);
    int k = tb ? (e / S::TN) : (e % TK);
    Bs[0][k][n] = (T)st.b[r].x;
    Bs[1][k][n] = (T)(cb ? -st.b[r].y : st.b[r].y);
  }
}

__device__ __forceinline__ bool next_ktile(const DevTerm* terms, int t_end, int& t, int& k0) {
  k0 += TK;
  if (k0 >= terms[t].K) {
    k0 = 0;
    ++t;
  }
  return t < t_end;
}

template <typename T, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void gemm_kernel(Bufs bufs, double* __restrict__ Cbase,
                                                           const DevTile* __restrict__ tiles,
                                                           const DevOut* __restrict__ outs,
                                                           const DevTerm* __restrict__ terms) {
  typedef Shape<WM, WN> S;
  typedef Mfma<T> F;
  __shared__ T As[2][TK][S::TM + PAD];
  __shared__ T Bs[2][TK][S::TN + PAD];
  const DevTile tl = tiles[blockIdx.x];
  const DevOut ob = outs[tl.out];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int li = lane & 15, lk = lane >> 4;

  typename F::acc_t accr[2][2], acci[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      accr[i][j] = typename F::acc_t{0, 0, 0, 0};
      acci[i][j] = typename F::acc_t{0, 0, 0, 0};
    }

  int t = ob.t_begin, k0 = 0;
  Stage<WM, WN> st;
  DevTerm cur;
  if (t < ob.t_end) {
    cur = terms[t];
    load_stage<WM, WN>(st, cur, bufs, tl.m0, tl.n0, ob.M, ob.N, k0, tid);
  }
  while (t < ob.t_end) {
    store_stage<T, WM, WN>(st, cur, As, Bs, tid);
    __syncthreads();
    int tn = t, kn = k0;
    bool more = next_ktile(terms, ob.t_end, tn, kn);
    DevTerm nxt;
    if (more) {
      nxt = terms[tn];
      load_stage<WM, WN>(st, nxt, bufs, tl.m0, tl.n0, ob.M, ob.N, kn, tid);
    }
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      T ar[2], ai[2], nai[2], br[2], bi[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        ar[i] = As[0][kk + lk][wm * 32 + i * 16 + li];
        ai[i] = As[1][kk + lk][wm * 32 + i * 16 + li];
        nai[i] = -ai[i];
        br[i] = Bs[0][kk + lk][wn * 32 + i * 16 + li];
        bi[i] = Bs[1][kk + lk][wn * 32 + i * 16 + li];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          accr[i][j] = F::op(ar[i], br[j], accr[i][j]);
          accr[i][j] = F::op(nai[i], bi[j], accr[i][j]);
          acci[i][j] = F::op(ar[i], bi[j], acci[i][j]);
          acci[i][j] = F::op(ai[i], br[j], acci[i][j]);
        }
    }
    __syncthreads();
    t = tn;
    k0 = kn;
    if (more) cur = nxt;
  }

  // direct (local) terms and the store
  double2* C = reinterpret_cast<double2*>(Cbase) + ob.c_off;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row = tl.m0 + wm * 32 + i * 16 + F::row(r, lk);
        int col = tl.n0 + wn * 32 + j * 16 + li;
        if (row < ob.M && col < ob.N) {
          double vr = accr[i][j][r], vi = acci[i][j][r];
          for (int d = ob.d_begin; d < ob.d_end; ++d) {
            const DevTerm dt = terms[d];
            const int64_t idx = (dt.ops & 1) ? (int64_t)col + (int64_t)row * dt.lda
                                             : (int64_t)row + (int64_t)col * dt.lda;
            const double2 x = (reinterpret_cast<const double2*>(bufs.p[dt.a_buf]) + dt.a_off)[idx];
            vr += dt.coef * x.x;
            vi += (dt.ops & 2) ? -dt.coef * x.y : dt.coef * x.y;
          }
          C[(int64_t)row + (int64_t)col * ob.ldc] = make_double2(vr, vi);
        }
      }
}

}  // namespace

Program::~Program() {
  if (!d_mem) return;
  if (pool) pool->free[cls].push_back(d_mem);
  else (void)hipFree(d_mem);
}

ProgPool::~ProgPool() {
  for (auto& kv : free)
    for (void* p : kv.second) (void)hipFree(p);
}

int default_tile_mode() {
  static int w = [] {
    const char* e = std::getenv("TDVP_TILE_MODE");
    int v = e ? std::atoi(e) : 2;
    return (v == 0 || v == 1) ? v : 2;
  }();
  return w;
}

// useful fraction of an M x N block tiled by t x t
static double tile_use(int M, int N, int t) {
  double pm = (double)((M + t - 1) / t * t), pn = (double)((N + t - 1) / t * t);
  return (double)M * (double)N / (pm * pn);
}

double tile_threshold() {
  static double v = [] {
    const char* e = std::getenv("TDVP_TILE_THR");
    return e ? std::atof(e) : 0.85;
  }();
  return v;
}

void Program::finalize() {
  tiles.clear();
  tile_mode = default_tile_mode();
  const double thr = tile_threshold();
  std::vector<DevTile> t64, t32;
  for (int o = 0; o < (int)outs.size(); ++o) {
    const DevOut& ob = outs[o];
    int64_t kc = 0;
    for (int t = ob.t_begin; t < ob.t_end; ++t) kc += (terms[t].K + TK - 1) / TK;
    int cost = (int)std::min<int64_t>(kc * TK + 4 * (ob.d_end - ob.d_begin), 0x7fffffff);
    // 64x64 tiles carry twice the arithmetic intensity of 32x32 ones: prefer
    // them unless their padding costs more than the threshold factor
    bool big = tile_mode == 2 || (tile_mode == 0 && tile_use(ob.M, ob.N, 64) >= thr * tile_use(ob.M, ob.N, 32));
    int tt = big ? 64 : 32;
    for (int m0 = 0; m0 < ob.M; m0 += tt)
      for (int n0 = 0; n0 < ob.N; n0 += tt) (big ? t64 : t32).push_back(DevTile{o, m0, n0, cost});
  }
  auto bycost = [](const DevTile& a, const DevTile& b) { return a.cost > b.cost; };
  std::stable_sort(t64.begin(), t64.end(), bycost);
  std::stable_sort(t32.begin(), t32.end(), bycost);
  n64 = (int)t64.size();
  tiles = t64;
  tiles.insert(tiles.end(), t32.begin(), t32.end());
}

DeviceBuffer::~DeviceBuffer() {
  if (p) (void)hipFree(p);
}

hipError_t DeviceBuffer::ensure(size_t n) {
  if (n <= bytes) return hipSuccess;
  if (p) {
    hipError_t e = hipFree(p);
    p = nullptr;
    bytes = 0;
    if (e != hipSuccess) return e;
  }
  size_t want = std::max(n, (size_t)256);
  hipError_t e = hipMalloc(&p, want);
  if (e == hipSuccess) bytes = want;
  return e;
}

int upload(tdvp_ctx* ctx, Program& p) {
  size_t bt = p.terms.size() * sizeof(DevTerm), bo = p.outs.size() * sizeof(DevOut),
         bl = p.tiles.size() * sizeof(DevTile);
  size_t total = bt + bo + bl + 3 * 256;
  if (p.d_mem) {
    if (p.pool) p.pool->free[p.cls].push_back(p.d_mem);
    else TDVP_HIP(ctx, hipFree(p.d_mem));
    p.d_mem = nullptr;
  }
  size_t cls = 4096;
  while (cls < total) cls <<= 1;
  p.pool = ctx->pool;
  p.cls = cls;
  auto& fl = ctx->pool->free[cls];
  if (!fl.empty()) {
    p.d_mem = fl.back();
    fl.pop_back();
  } else {
    TDVP_HIP(ctx, hipMalloc(&p.d_mem, cls));
  }
  char* base = (char*)p.d_mem;
  auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
  p.d_terms = (DevTerm*)base;
  p.d_outs = (DevOut*)(base + align(bt));
  p.d_tiles = (DevTile*)(base + align(bt) + align(bo));
  // stage through pinned memory; wait for the previous upload before reuse
  if (ctx->upload_done) TDVP_HIP(ctx, hipEventSynchronize(ctx->upload_done));
  if (ctx->pinned_bytes < total) {
    if (ctx->pinned) TDVP_HIP(ctx, hipHostFree(ctx->pinned));
    ctx->pinned = nullptr;
    ctx->pinned_bytes = 0;
    TDVP_HIP(ctx, hipHostMalloc(&ctx->pinned, total));
    ctx->pinned_bytes = total;
  }
  char* h = (char*)ctx->pinned;
  if (bt) std::memcpy(h, p.terms.data(), bt);
  if (bo) std::memcpy(h + align(bt), p.outs.data(), bo);
  if (bl) std::memcpy(h + align(bt) + align(bo), p.tiles.data(), bl);
  TDVP_HIP(ctx, hipMemcpyAsync(p.d_mem, h, align(bt) + align(bo) + bl, hipMemcpyHostToDevice, ctx->stream));
  if (!ctx->upload_done) TDVP_HIP(ctx, hipEventCreateWithFlags(&ctx->upload_done, hipEventDisableTiming));
  TDVP_HIP(ctx, hipEventRecord(ctx->upload_done, ctx->stream));
  return TDVP_OK;
}

std::shared_ptr<Program> cache_get(tdvp_ctx* ctx, uint64_t key) {
  for (auto it = ctx->cache.begin(); it != ctx->cache.end(); ++it)
    if (it->first == key) {
      auto p = it->second;
      ctx->cache.splice(ctx->cache.begin(), ctx->cache, it);
      return p;
    }
  return nullptr;
}

void cache_put(tdvp_ctx* ctx, uint64_t key, std::shared_ptr<Program> p) {
  ctx->cache.emplace_front(key, std::move(p));
  while (ctx->cache.size() > 24) ctx->cache.pop_back();
}

int launch_gemm(tdvp_ctx* ctx, const Program& p, const Bufs& bufs, double* C, int precision) {
  if (p.tiles.empty()) return TDVP_OK;
  const int n32 = (int)p.tiles.size() - p.n64;
  const DevTile* t32 = p.d_tiles + p.n64;
  if (p.n64 > 0) {
    if (precision == TDVP_FP32)
      hipLaunchKernelGGL((gemm_kernel<float, 2, 2>), dim3(p.n64), dim3(256), 0, ctx->stream, bufs, C, p.d_tiles,
                         p.d_outs, p.d_terms);
    else
      hipLaunchKernelGGL((gemm_kernel<double, 2, 2>), dim3(p.n64), dim3(256), 0, ctx->stream, bufs, C, p.d_tiles,
                         p.d_outs, p.d_terms);
  }
  if (n32 > 0) {
    if (precision == TDVP_FP32)
      hipLaunchKernelGGL((gemm_kernel<float, 1, 1>), dim3(n32), dim3(64), 0, ctx->stream, bufs, C, t32, p.d_outs,
                         p.d_terms);
    else
      hipLaunchKernelGGL((gemm_kernel<double, 1, 1>), dim3(n32), dim3(64), 0, ctx->stream, bufs, C, t32, p.d_outs,
                         p.d_terms);
  }
  TDVP_HIP(ctx, hipGetLastError());
  return TDVP_OK;
}

}  // namespace tdvp

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
#include <cmath>
#include <map>
#include <cstdlib>
#include <cstring>

#include "common.hpp"
#include "ctx.hpp"

namespace tdvp {

namespace {

constexpr int PAD = 2;
// K depth of one staged step: 16 for FP64 tiles, 32 for FP32 ones (measured:
// FP64 loses occupancy at 32, FP32 gains from the longer step)
template <typename T>
struct KStep {
  static constexpr int value = sizeof(T) == 8 ? 16 : 32;
};
// host-side stepping of K chains (cost model, split points): a multiple of every KStep
constexpr int kHostKStep = 32;

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
template <typename T, int WM, int WN>
struct Shape {
  static constexpr int TK = KStep<T>::value;
  static constexpr int TM = 32 * WM, TN = 32 * WN, NT = 64 * WM * WN;
  static constexpr int NA = TM * TK / NT, NB = TK * TN / NT;   // elements per thread
};

template <typename T, int WM, int WN>
struct Stage {
  double2 a[Shape<T, WM, WN>::NA], b[Shape<T, WM, WN>::NB];
};

// Load this thread's A and B elements of the K-tile k0 of term tm (coalesced:
// consecutive threads follow the contiguous dimension of each operand).
template <typename T, int WM, int WN, bool SH>
__device__ __forceinline__ void load_stage(Stage<T, WM, WN>& st, const DevTerm& tm, const Bufs& bufs, int m0, int n0,
                                           int M, int N, int k0, int tid) {
  typedef Shape<T, WM, WN> S;
  constexpr int TK = S::TK;
  const double2* A = reinterpret_cast<const double2*>(bufs.p[tm.a_buf]) + tm.a_off;
  const double2* B = reinterpret_cast<const double2*>(bufs.p[tm.b_buf]) + tm.b_off;
  const bool ta = tm.ops & 1, tb = tm.ops & 4;
  // diagonal shifts only where this K step meets the diagonal (uniform test)
  const bool shA = SH && (tm.ops & 16) && m0 < k0 + TK && k0 < m0 + S::TM;
  const bool shB = SH && (tm.ops & 32) && n0 < k0 + TK && k0 < n0 + S::TN;
#pragma unroll
  for (int r = 0; r < S::NA; ++r) {
    int e = tid + S::NT * r;
    int m = ta ? (e / TK) : (e % S::TM);
    int k = ta ? (e % TK) : (e / S::TM);
    int gm = m0 + m, gk = k0 + k;
    double2 v = make_double2(0.0, 0.0);
    if (gm < M && gk < tm.K) {
      v = ta ? A[(int64_t)gk + (int64_t)gm * tm.lda] : A[(int64_t)gm + (int64_t)gk * tm.lda];
      if (shA && gm == gk) v.x -= bufs.shift[0];
    }
    st.a[r] = v;
  }
#pragma unroll
  for (int r = 0; r < S::NB; ++r) {
    int e = tid + S::NT * r;
    int n = tb ? (e % S::TN) : (e / TK);
    int k = tb ? (e / S::TN) : (e % TK);
    int gn = n0 + n, gk = k0 + k;
    double2 v = make_double2(0.0, 0.0);
    if (gn < N && gk < tm.K) {
      v = tb ? B[(int64_t)gn + (int64_t)gk * tm.ldb] : B[(int64_t)gk + (int64_t)gn * tm.ldb];
      if (shB && gn == gk) v.x -= bufs.shift[1];
    }
    st.b[r] = v;
  }
}

template <typename T, int WM, int WN>
__device__ __forceinline__ void store_stage(const Stage<T, WM, WN>& st, const DevTerm& tm,
                                            T (*As)[Shape<T, WM, WN>::TK][Shape<T, WM, WN>::TM + PAD],
                                            T (*Bs)[Shape<T, WM, WN>::TK][Shape<T, WM, WN>::TN + PAD], int tid) {
  typedef Shape<T, WM, WN> S;
  constexpr int TK = S::TK;
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

template <typename T>
__device__ __forceinline__ void next_ktile(const DevTerm* terms, int& t, int& k0) {
  k0 += KStep<T>::value;
  if (k0 >= terms[t].K) {
    k0 = 0;
    ++t;
  }
}

__device__ __forceinline__ bool before(int t, int k0, int t1, int k1) { return t < t1 || (t == t1 && k0 < k1); }

// Partial tiles are stored TM_MAX x TN_MAX, column-major, whatever the tile shape.
constexpr int kSlotDim = 64;

template <typename T, int WM, int WN, bool SH>
__device__ __forceinline__ void gemm_body(const Bufs& bufs, double* __restrict__ Cbase,
                                          double2* __restrict__ part, const DevTile* __restrict__ tiles,
                                          const DevOut* __restrict__ outs, const DevTerm* __restrict__ terms,
                                          int tile) {
  typedef Shape<T, WM, WN> S;
  typedef Mfma<T> F;
  constexpr int TK = S::TK;
  __shared__ T As[2][TK][S::TM + PAD];
  __shared__ T Bs[2][TK][S::TN + PAD];
  const DevTile tl = tiles[tile];
  const DevOut ob = outs[tl.out];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int li = lane & 15, lk = lane >> 4;
  // 16 x 16 sub-blocks of this wave that lie inside the output (wave-uniform):
  // the matrix instructions of the others are skipped
  bool rv[2], cv[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    rv[i] = tl.m0 + wm * 32 + i * 16 < ob.M;
    cv[i] = tl.n0 + wn * 32 + i * 16 < ob.N;
  }

  typename F::acc_t accr[2][2], acci[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      accr[i][j] = typename F::acc_t{0, 0, 0, 0};
      acci[i][j] = typename F::acc_t{0, 0, 0, 0};
    }

  int t = tl.t0, k0 = tl.k0;
  Stage<T, WM, WN> st;
  DevTerm cur;
  if (before(t, k0, tl.t1, tl.k1)) {
    cur = terms[t];
    load_stage<T, WM, WN, SH>(st, cur, bufs, tl.m0, tl.n0, ob.M, ob.N, k0, tid);
  }
  while (before(t, k0, tl.t1, tl.k1)) {
    store_stage<T, WM, WN>(st, cur, As, Bs, tid);
    __syncthreads();
    const int krem = cur.K - k0;   // valid depth of this K step
    int tn = t, kn = k0;
    next_ktile<T>(terms, tn, kn);
    const bool more = before(tn, kn, tl.t1, tl.k1);
    DevTerm nxt;
    if (more) {
      nxt = (tn == t) ? cur : terms[tn];   // the term is reloaded only when it changes
      load_stage<T, WM, WN, SH>(st, nxt, bufs, tl.m0, tl.n0, ob.M, ob.N, kn, tid);
    }
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      if (kk < krem) {
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
          for (int j = 0; j < 2; ++j)
            if (rv[i] && cv[j]) {
              accr[i][j] = F::op(ar[i], br[j], accr[i][j]);
              accr[i][j] = F::op(nai[i], bi[j], accr[i][j]);
              acci[i][j] = F::op(ar[i], bi[j], acci[i][j]);
              acci[i][j] = F::op(ai[i], br[j], acci[i][j]);
            }
      }
    }
    __syncthreads();
    t = tn;
    k0 = kn;
    if (more) cur = nxt;
  }

  if (tl.slot >= 0) {   // partial sum of a split chain
    double2* P = part + (int64_t)tl.slot * kSlotDim * kSlotDim;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int lr = wm * 32 + i * 16 + F::row(r, lk);
          int lc = wn * 32 + j * 16 + li;
          if (tl.m0 + lr < ob.M && tl.n0 + lc < ob.N)
            P[lr + lc * kSlotDim] = make_double2((double)accr[i][j][r], (double)acci[i][j][r]);
        }
    return;
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
            if (!SH && (dt.ops & 48)) continue;   // compensation of shifts not applied
            const int64_t idx = (dt.ops & 1) ? (int64_t)col + (int64_t)row * dt.lda
                                             : (int64_t)row + (int64_t)col * dt.lda;
            const double2 x = (reinterpret_cast<const double2*>(bufs.p[dt.a_buf]) + dt.a_off)[idx];
            double c = dt.coef;
            if (SH && (dt.ops & 16)) c *= bufs.shift[0];
            if (SH && (dt.ops & 32)) c *= bufs.shift[1];
            vr += c * x.x;
            vi += (dt.ops & 2) ? -c * x.y : c * x.y;
          }
          if (bufs.bad && !(isfinite(vr) && isfinite(vi))) *bufs.bad = 1;
          C[(int64_t)row + (int64_t)col * ob.ldc] = make_double2(vr, vi);
        }
      }
}

// ---------------------------------------------------------------------------
// FP64 wave tiles: one 32x32 output tile per wave, four independent waves per
// workgroup, operands loaded by each lane straight into the registers the
// matrix instruction reads (no LDS staging, no barriers), two K steps of 4
// ahead of the one being multiplied.  A wave whose tile is a ragged edge
// spends its time only on its own 16x16 sub-blocks, and no wave waits for
// another.  Every output element sees the same products in the same order as
// in gemm_body<double, WM, WN> (K steps of 4 with lane group l / 16 holding
// k + l / 16, the term coefficient and conjugations applied to the same
// values, the same matrix instruction sequence per 16x16 sub-block), so the
// results are bit-identical to every other FP64 tiling.
struct WPos {
  int t, k;   // term, K offset (a multiple of 4) inside it
};

template <int MR, int MC>
struct WStage {
  double2 a[MR], b[MC];
  double c;
  int k;          // the step's K offset
  bool ca, cb;
  bool sha, shb;  // reduced precision: the energy shift on the diagonal of A (B)
};

// Steps of a chain: K offsets 0, 4, ... below K of every term in [t0, t1).
__device__ __forceinline__ int wave_steps(const DevTerm* __restrict__ terms, int t0, int t1) {
  int n = 0;
  for (int t = t0; t < t1; ++t) n += (terms[t].K + 3) >> 2;
  return n;
}

// First step at or after p (terms with K = 0 have none); p.t == t1 at the end.
__device__ __forceinline__ void wave_settle(const DevTerm* __restrict__ terms, WPos& p, int t1) {
  while (p.t < t1 && p.k >= terms[p.t].K) {
    p.k = 0;
    ++p.t;
  }
}

// The next step, or p itself when p is the chain's last step (the loads of the
// pipeline's lookahead then re-read valid data that is never used).
__device__ __forceinline__ void wave_next(const DevTerm* __restrict__ terms, WPos& p, int t1) {
  WPos q{p.t, p.k + 4};
  wave_settle(terms, q, t1);
  if (q.t < t1) p = q;
}

// Lanes outside the block load this zero instead of an operand element, so
// that every load is issued unconditionally and its value is used as loaded.
// Both addresses are global-memory pointers (a select of generic pointers
// would turn the loads into flat ones, which the scalar loads' waits then
// also wait for).
__device__ const double2 kZero2 = {0.0, 0.0};
#if defined(__HIP_DEVICE_COMPILE__)
typedef const __attribute__((address_space(1))) double2* gptr2;
#else
typedef const double2* gptr2;   // the host pass only parses the device code
#endif

template <bool SH, int MR, int MC>
__device__ __forceinline__ void wave_load(WStage<MR, MC>& s, const DevTerm* __restrict__ terms, const WPos& p,
                                          const Bufs& bufs, int m0, int n0, int M, int N, int li, int lk) {
  const DevTerm& tm = terms[p.t];
  s.c = tm.coef;
  s.k = p.k;
  s.ca = tm.ops & 2;
  s.cb = tm.ops & 8;
  s.sha = SH && (tm.ops & 16);
  s.shb = SH && (tm.ops & 32);
  const gptr2 A = (gptr2)(reinterpret_cast<const double2*>(bufs.p[tm.a_buf]) + tm.a_off);
  const gptr2 B = (gptr2)(reinterpret_cast<const double2*>(bufs.p[tm.b_buf]) + tm.b_off);
  const gptr2 Z = (gptr2)&kZero2;
  const bool ta = tm.ops & 1, tb = tm.ops & 4;
  const int k = p.k + lk;
  // element (row, k) of A at row * sa_r + k * sa_k, (k, col) of B at k * sb_k + col * sb_c
  const int64_t sa_r = ta ? tm.lda : 1, sa_k = ta ? 1 : tm.lda;
  const int64_t sb_k = tb ? tm.ldb : 1, sb_c = tb ? 1 : tm.ldb;
  const bool kin = k < tm.K;
#pragma unroll
  for (int i = 0; i < MR; ++i) {
    const int gm = m0 + i * 16 + li;
    const gptr2 at = A + ((int64_t)gm * sa_r + (int64_t)k * sa_k);
    s.a[i] = *((kin && gm < M) ? at : Z);
  }
#pragma unroll
  for (int j = 0; j < MC; ++j) {
    const int gn = n0 + j * 16 + li;
    const gptr2 at = B + ((int64_t)k * sb_k + (int64_t)gn * sb_c);
    s.b[j] = *((kin && gn < N) ? at : Z);
  }
}

// The products of one step.  Values as the LDS-staged kernel stages them:
// the shift subtracted on the diagonal, then coefficient and conjugation in
// FP64, then the conversion to T.
template <typename T, bool SH, int MR, int MC>
__device__ __forceinline__ void wave_mma(const WStage<MR, MC>& s, typename Mfma<T>::acc_t (&accr)[2][2],
                                         typename Mfma<T>::acc_t (&acci)[2][2], const int (&gm)[MR],
                                         const int (&gn)[MC], int lk, double sh0, double sh1) {
  T ar[MR], ai[MR], nai[MR], br[MC], bi[MC];
  const int k = s.k + lk;
#pragma unroll
  for (int i = 0; i < MR; ++i) {
    double x = s.a[i].x;
    if (SH && s.sha && gm[i] == k) x -= sh0;
    ar[i] = (T)(s.c * x);
    ai[i] = (T)(s.ca ? -s.c * s.a[i].y : s.c * s.a[i].y);
    nai[i] = -ai[i];
  }
#pragma unroll
  for (int j = 0; j < MC; ++j) {
    double x = s.b[j].x;
    if (SH && s.shb && gn[j] == k) x -= sh1;
    br[j] = (T)x;
    bi[j] = (T)(s.cb ? -s.b[j].y : s.b[j].y);
  }
#pragma unroll
  for (int i = 0; i < MR; ++i)
#pragma unroll
    for (int j = 0; j < MC; ++j) {
      accr[i][j] = Mfma<T>::op(ar[i], br[j], accr[i][j]);
      accr[i][j] = Mfma<T>::op(nai[i], bi[j], accr[i][j]);
      acci[i][j] = Mfma<T>::op(ar[i], bi[j], acci[i][j]);
      acci[i][j] = Mfma<T>::op(ai[i], br[j], acci[i][j]);
    }
}

// The K chain of one wave tile with MR x MC of its 16x16 sub-blocks inside
// the output: three register stages, loads two steps ahead of the products.
template <typename T, bool SH, int MR, int MC>
__device__ __forceinline__ void wave_chain(const Bufs& bufs, const DevTerm* __restrict__ terms, const DevTile& tl,
                                           const DevOut& ob, int li, int lk, typename Mfma<T>::acc_t (&accr)[2][2],
                                           typename Mfma<T>::acc_t (&acci)[2][2]) {
  const int t1 = tl.t1;
  const int n = wave_steps(terms, tl.t0, t1);
  if (n == 0) return;
  int gm[MR], gn[MC];
#pragma unroll
  for (int i = 0; i < MR; ++i) gm[i] = tl.m0 + i * 16 + li;
#pragma unroll
  for (int j = 0; j < MC; ++j) gn[j] = tl.n0 + j * 16 + li;
  const double sh0 = SH ? bufs.shift[0] : 0.0, sh1 = SH ? bufs.shift[1] : 0.0;
  WPos p{tl.t0, 0};
  wave_settle(terms, p, t1);
  WStage<MR, MC> s0, s1, s2;
  wave_load<SH>(s0, terms, p, bufs, tl.m0, tl.n0, ob.M, ob.N, li, lk);
  wave_next(terms, p, t1);
  wave_load<SH>(s1, terms, p, bufs, tl.m0, tl.n0, ob.M, ob.N, li, lk);
  wave_next(terms, p, t1);
  int i = 0;
  for (; i + 3 <= n; i += 3) {   // steps i, i+1, i+2 are all in the chain
    wave_load<SH>(s2, terms, p, bufs, tl.m0, tl.n0, ob.M, ob.N, li, lk);
    wave_next(terms, p, t1);
    wave_mma<T, SH>(s0, accr, acci, gm, gn, lk, sh0, sh1);
    wave_load<SH>(s0, terms, p, bufs, tl.m0, tl.n0, ob.M, ob.N, li, lk);
    wave_next(terms, p, t1);
    wave_mma<T, SH>(s1, accr, acci, gm, gn, lk, sh0, sh1);
    wave_load<SH>(s1, terms, p, bufs, tl.m0, tl.n0, ob.M, ob.N, li, lk);
    wave_next(terms, p, t1);
    wave_mma<T, SH>(s2, accr, acci, gm, gn, lk, sh0, sh1);
  }
  if (i < n) wave_mma<T, SH>(s0, accr, acci, gm, gn, lk, sh0, sh1);
  if (i + 1 < n) wave_mma<T, SH>(s1, accr, acci, gm, gn, lk, sh0, sh1);
}

template <typename T, bool SH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void heff_gemm_wave(
    Bufs bufs, double* __restrict__ Cbase, const DevTile* __restrict__ tiles, int ntiles,
    const DevOut* __restrict__ outs, const DevTerm* __restrict__ terms) {
  typedef typename Mfma<T>::acc_t acc_t;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tile = blockIdx.x * 4 + wave;
  if (tile >= ntiles) return;   // whole waves only: nothing below synchronises the workgroup
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const DevTile tl = tiles[tile];
  const DevOut ob = outs[tl.out];
  acc_t accr[2][2], acci[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      accr[i][j] = acc_t{0, 0, 0, 0};
      acci[i][j] = acc_t{0, 0, 0, 0};
    }
  // whole chains only (wave tiles are never split): terms [t0, t1) from K = 0
  const bool r2 = tl.m0 + 16 < ob.M, c2 = tl.n0 + 16 < ob.N;
  if (r2 && c2) wave_chain<T, SH, 2, 2>(bufs, terms, tl, ob, li, lk, accr, acci);
  else if (r2) wave_chain<T, SH, 2, 1>(bufs, terms, tl, ob, li, lk, accr, acci);
  else if (c2) wave_chain<T, SH, 1, 2>(bufs, terms, tl, ob, li, lk, accr, acci);
  else wave_chain<T, SH, 1, 1>(bufs, terms, tl, ob, li, lk, accr, acci);
  // direct (local) terms and the store, as in gemm_body
  double2* C = reinterpret_cast<double2*>(Cbase) + ob.c_off;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row = tl.m0 + i * 16 + Mfma<T>::row(r, lk);
        int col = tl.n0 + j * 16 + li;
        if (row < ob.M && col < ob.N) {
          double vr = accr[i][j][r], vi = acci[i][j][r];
          for (int d = ob.d_begin; d < ob.d_end; ++d) {
            const DevTerm dt = terms[d];
            if (!SH && (dt.ops & 48)) continue;   // compensation of shifts not applied
            const int64_t idx = (dt.ops & 1) ? (int64_t)col + (int64_t)row * dt.lda
                                             : (int64_t)row + (int64_t)col * dt.lda;
            const double2 x = (reinterpret_cast<const double2*>(bufs.p[dt.a_buf]) + dt.a_off)[idx];
            double c = dt.coef;
            if (SH && (dt.ops & 16)) c *= bufs.shift[0];
            if (SH && (dt.ops & 32)) c *= bufs.shift[1];
            vr += c * x.x;
            vi += (dt.ops & 2) ? -c * x.y : c * x.y;
          }
          if (bufs.bad && !(isfinite(vr) && isfinite(vi))) *bufs.bad = 1;
          C[(int64_t)row + (int64_t)col * ob.ldc] = make_double2(vr, vi);
        }
      }
}

// ---------------------------------------------------------------------------
// Split-BF16 products (Ozaki-style).  Every operand value a (real and
// imaginary parts separately) is cut into three bfloat16 slices
// a = a1 + a2 + a3 (each the round-to-nearest of the remainder, in FP32), and
// each real product keeps the six slice products whose slice indices sum to
// at most four, accumulated in FP32 on v_mfma_f32_16x16x32_bf16.  Lane layout
// of that instruction: A[i][k] for i = lane % 16 and k = 8 (lane / 16) .. +7
// (one 16-byte vector), B[k][j] likewise with j = lane % 16, D as the FP32
// 16x16x4 one.
//
// The slicing is done once per operand buffer and launch by a streaming
// kernel (slice_records), not per tile: each complex element becomes one
// 16-byte record, dword s (s = 0, 1, 2) holding slice s of the real part in
// its low and of the imaginary part in its high half (dword 3 zero).  The
// energy shift of the block-Hamiltonian environment blocks is applied to
// their diagonals in the records (slice_fix_diag).  The tile loop only loads
// records, regroups their halves into per-slice LDS rows of K = 32
// contiguous values (conjugation = a sign flip of the imaginary halves) and
// issues matrix instructions.  The term coefficient multiplies a term group's
// FP32 partial sum when the coefficient changes along the K chain.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int TKB = 32, PADB = 8;

struct Slices {
  const uint4* p[kMaxBufs];   // records of buffer b, p[b][e - lo[b]] for element e
  int64_t lo[kMaxBufs];
};

__device__ __forceinline__ uint32_t bf16_bits(float f) {
  return (uint32_t)__builtin_bit_cast(unsigned short, (__bf16)f);
}
__device__ __forceinline__ float bf16_value(uint32_t bits) { return __uint_as_float(bits << 16); }

__device__ __forceinline__ void slice3_bits(double v, uint32_t& s1, uint32_t& s2, uint32_t& s3) {
  const float f = (float)v;
  s1 = bf16_bits(f);
  const float r1 = f - bf16_value(s1);
  s2 = bf16_bits(r1);
  s3 = bf16_bits(r1 - bf16_value(s2));
}

__device__ __forceinline__ uint4 make_record(double2 v) {
  uint32_t r1, r2, r3, i1, i2, i3;
  slice3_bits(v.x, r1, r2, r3);
  slice3_bits(v.y, i1, i2, i3);
  return make_uint4(r1 | (i1 << 16), r2 | (i2 << 16), r3 | (i3 << 16), 0u);
}

__global__ __launch_bounds__(256) void slice_records(const double2* __restrict__ src, uint4* __restrict__ dst,
                                                     int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
    dst[e] = make_record(src[e]);
}

// Records of the diagonals of the listed blocks (meta: offset, dimension,
// weight triplets) re-made from E - shift: one workgroup per block.  Only
// elements inside the sliced range [lo, hi) have records (a listed block that
// no product reads may lie outside it).
__global__ __launch_bounds__(256) void slice_fix_diag(const double2* __restrict__ E, uint4* __restrict__ dst,
                                                      int64_t lo, int64_t hi, const int64_t* __restrict__ meta,
                                                      const double* __restrict__ shift) {
  const int64_t off = meta[3 * blockIdx.x], d = meta[3 * blockIdx.x + 1];
  const double e0 = *shift;
  for (int64_t i = threadIdx.x; i < d; i += 256) {
    const int64_t e = off + i * (d + 1);
    if (e < lo || e >= hi) continue;
    double2 v = E[e];
    v.x -= e0;
    dst[e - lo] = make_record(v);
  }
}

__device__ __forceinline__ uint32_t rec_word(const uint4& r, int s) { return s == 0 ? r.x : s == 1 ? r.y : r.z; }

template <bool SH>
__device__ __forceinline__ void gemm_body_b3(const Bufs& bufs, const Slices& sl, double* __restrict__ Cbase,
                                             double2* __restrict__ part, const DevTile* __restrict__ tiles,
                                             const DevOut* __restrict__ outs, const DevTerm* __restrict__ terms) {
  constexpr int TM = 64, TN = 64;
  typedef f32x4 acc_t;
  __shared__ __attribute__((aligned(16))) __bf16 As[3][2][TM][TKB + PADB];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[3][2][TN][TKB + PADB];
  const DevTile tl = tiles[blockIdx.x];
  const DevOut ob = outs[tl.out];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / 2, wn = wave % 2;
  const int li = lane & 15, lk = lane >> 4;
  bool rv[2], cv[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    rv[i] = tl.m0 + wm * 32 + i * 16 < ob.M;
    cv[i] = tl.n0 + wn * 32 + i * 16 < ob.N;
  }
  // accr/acci: the tile's sum; tr/ti: the partial sum of the current group of
  // consecutive terms with one coefficient (ccur)
  acc_t accr[2][2], acci[2][2], tr[2][2], ti[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      accr[i][j] = acc_t{0, 0, 0, 0};
      acci[i][j] = acc_t{0, 0, 0, 0};
      tr[i][j] = acc_t{0, 0, 0, 0};
      ti[i][j] = acc_t{0, 0, 0, 0};
    }
  auto flush = [&](double c) {
    const float cf = (float)c;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        accr[i][j] += cf * tr[i][j];
        acci[i][j] += cf * ti[i][j];
        tr[i][j] = acc_t{0, 0, 0, 0};
        ti[i][j] = acc_t{0, 0, 0, 0};
      }
  };
  // staging: this thread owns row sr of the A and B tiles and 8 consecutive k;
  // the records of the next K step are loaded into registers while the
  // matrix instructions of the current one run
  const int sr = tid % 64, kg = tid / 64;
  int t = tl.t0, k0 = tl.k0;
  uint4 ra[8], rb[8];
  auto load_records = [&](const DevTerm& tm, int kk0) {
    const uint4* A = sl.p[tm.a_buf] + (tm.a_off - sl.lo[tm.a_buf]);
    const uint4* B = sl.p[tm.b_buf] + (tm.b_off - sl.lo[tm.b_buf]);
    const bool ta = tm.ops & 1, tb = tm.ops & 4;
    const int gm = tl.m0 + sr, gn = tl.n0 + sr;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int gk = kk0 + 8 * kg + q;
      ra[q] = make_uint4(0u, 0u, 0u, 0u);
      rb[q] = make_uint4(0u, 0u, 0u, 0u);
      if (gm < ob.M && gk < tm.K) ra[q] = ta ? A[(int64_t)gk + (int64_t)gm * tm.lda] : A[(int64_t)gm + (int64_t)gk * tm.lda];
      if (gn < ob.N && gk < tm.K) rb[q] = tb ? B[(int64_t)gn + (int64_t)gk * tm.ldb] : B[(int64_t)gk + (int64_t)gn * tm.ldb];
    }
  };
  DevTerm cur;
  double ccur = 0.0;
  if (before(t, k0, tl.t1, tl.k1)) {
    cur = terms[t];
    ccur = cur.coef;
    load_records(cur, k0);
  }
  while (before(t, k0, tl.t1, tl.k1)) {
    if (cur.coef != ccur) {   // uniform: a new coefficient group
      flush(ccur);
      ccur = cur.coef;
    }
    {
      const uint32_t sa = (cur.ops & 2) ? 0x80008000u : 0u, sb = (cur.ops & 8) ? 0x80008000u : 0u;
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        uint4 are, aim, bre, bim;
        uint32_t* pare = reinterpret_cast<uint32_t*>(&are);
        uint32_t* paim = reinterpret_cast<uint32_t*>(&aim);
        uint32_t* pbre = reinterpret_cast<uint32_t*>(&bre);
        uint32_t* pbim = reinterpret_cast<uint32_t*>(&bim);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint32_t a0 = rec_word(ra[2 * j], s), a1 = rec_word(ra[2 * j + 1], s);
          const uint32_t b0 = rec_word(rb[2 * j], s), b1 = rec_word(rb[2 * j + 1], s);
          pare[j] = (a0 & 0xffffu) | (a1 << 16);
          paim[j] = ((a0 >> 16) | (a1 & 0xffff0000u)) ^ sa;
          pbre[j] = (b0 & 0xffffu) | (b1 << 16);
          pbim[j] = ((b0 >> 16) | (b1 & 0xffff0000u)) ^ sb;
        }
        *reinterpret_cast<uint4*>(&As[s][0][sr][8 * kg]) = are;
        *reinterpret_cast<uint4*>(&As[s][1][sr][8 * kg]) = aim;
        *reinterpret_cast<uint4*>(&Bs[s][0][sr][8 * kg]) = bre;
        *reinterpret_cast<uint4*>(&Bs[s][1][sr][8 * kg]) = bim;
      }
    }
    __syncthreads();
    int tn = t, kn = k0 + TKB;
    if (kn >= cur.K) {
      kn = 0;
      ++tn;
    }
    const bool more = before(tn, kn, tl.t1, tl.k1);
    DevTerm nxt;
    if (more) {
      nxt = (tn == t) ? cur : terms[tn];   // the term is reloaded only when it changes
      load_records(nxt, kn);
    }
    // B fragments of both column blocks once, then A per row block
    bf16x8 br[2][3], bi[2][3];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        br[j][s] = *reinterpret_cast<const bf16x8*>(&Bs[s][0][wn * 32 + j * 16 + li][8 * lk]);
        bi[j][s] = *reinterpret_cast<const bf16x8*>(&Bs[s][1][wn * 32 + j * 16 + li][8 * lk]);
      }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      if (!rv[i]) continue;
      bf16x8 ar[3], ai[3], nai[3];
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        ar[s] = *reinterpret_cast<const bf16x8*>(&As[s][0][wm * 32 + i * 16 + li][8 * lk]);
        ai[s] = *reinterpret_cast<const bf16x8*>(&As[s][1][wm * 32 + i * 16 + li][8 * lk]);
        const uint4 u = *reinterpret_cast<const uint4*>(&ai[s]);
        const uint4 nu = make_uint4(u.x ^ 0x80008000u, u.y ^ 0x80008000u, u.z ^ 0x80008000u, u.w ^ 0x80008000u);
        nai[s] = *reinterpret_cast<const bf16x8*>(&nu);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        if (!cv[j]) continue;
        // slice pairs (0,0) (0,1) (1,0) (0,2) (1,1) (2,0), smallest first
#pragma unroll
        for (int pp = 5; pp >= 0; --pp) {
          const int x = pp == 0 ? 0 : pp == 1 ? 0 : pp == 2 ? 1 : pp == 3 ? 0 : pp == 4 ? 1 : 2;
          const int y = pp == 0 ? 0 : pp == 1 ? 1 : pp == 2 ? 0 : pp == 3 ? 2 : pp == 4 ? 1 : 0;
          tr[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar[x], br[j][y], tr[i][j], 0, 0, 0);
          ti[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar[x], bi[j][y], ti[i][j], 0, 0, 0);
          tr[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nai[x], bi[j][y], tr[i][j], 0, 0, 0);
          ti[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[x], br[j][y], ti[i][j], 0, 0, 0);
        }
      }
    }
    __syncthreads();
    t = tn;
    k0 = kn;
    if (more) cur = nxt;
  }
  flush(ccur);

  if (tl.slot >= 0) {
    double2* P = part + (int64_t)tl.slot * kSlotDim * kSlotDim;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int lr = wm * 32 + i * 16 + 4 * lk + r;
          int lc = wn * 32 + j * 16 + li;
          if (tl.m0 + lr < ob.M && tl.n0 + lc < ob.N)
            P[lr + lc * kSlotDim] = make_double2((double)accr[i][j][r], (double)acci[i][j][r]);
        }
    return;
  }
  double2* C = reinterpret_cast<double2*>(Cbase) + ob.c_off;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row = tl.m0 + wm * 32 + i * 16 + 4 * lk + r;
        int col = tl.n0 + wn * 32 + j * 16 + li;
        if (row < ob.M && col < ob.N) {
          double vr = accr[i][j][r], vi = acci[i][j][r];
          for (int d = ob.d_begin; d < ob.d_end; ++d) {
            const DevTerm dt = terms[d];
            if (!SH && (dt.ops & 48)) continue;
            const int64_t idx = (dt.ops & 1) ? (int64_t)col + (int64_t)row * dt.lda
                                             : (int64_t)row + (int64_t)col * dt.lda;
            const double2 xv = (reinterpret_cast<const double2*>(bufs.p[dt.a_buf]) + dt.a_off)[idx];
            double cc = dt.coef;
            if (SH && (dt.ops & 16)) cc *= bufs.shift[0];
            if (SH && (dt.ops & 32)) cc *= bufs.shift[1];
            vr += cc * xv.x;
            vi += (dt.ops & 2) ? -cc * xv.y : cc * xv.y;
          }
          if (bufs.bad && !(isfinite(vr) && isfinite(vi))) *bufs.bad = 1;
          C[(int64_t)row + (int64_t)col * ob.ldc] = make_double2(vr, vi);
        }
      }
}

template <bool SH>
__global__ __launch_bounds__(256) void heff_gemm_b3(Bufs bufs, Slices sl, double* __restrict__ C,
                                                    double2* __restrict__ part, const DevTile* __restrict__ tiles,
                                                    const DevOut* __restrict__ outs,
                                                    const DevTerm* __restrict__ terms) {
  gemm_body_b3<SH>(bufs, sl, C, part, tiles, outs, terms);
}
template <bool SH>
__global__ __launch_bounds__(256) void block_gemm_b3(Bufs bufs, Slices sl, double* __restrict__ C,
                                                     double2* __restrict__ part, const DevTile* __restrict__ tiles,
                                                     const DevOut* __restrict__ outs,
                                                     const DevTerm* __restrict__ terms) {
  gemm_body_b3<SH>(bufs, sl, C, part, tiles, outs, terms);
}

// Diagonal shifts of a reduced-precision launch: out[s] = sum_b w_b tr(E_b) /
// sum_b w_b d_b over the listed diagonal blocks of operand buffer 1 + s.
// First pass: one workgroup per listed block writes w_b tr(E_b) and w_b d_b.
__global__ __launch_bounds__(256) void env_shift_parts(Bufs bufs, const int64_t* __restrict__ meta, int n0,
                                                       double2* __restrict__ part) {
  const int b = blockIdx.x;
  const double2* E = reinterpret_cast<const double2*>(bufs.p[b < n0 ? 1 : 2]);
  const int64_t off = meta[3 * b], d = meta[3 * b + 1];
  const double w = (double)meta[3 * b + 2];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < d; i += 256) s += E[off + i * (d + 1)].x;
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[b] = make_double2(w * red[0], w * (double)d);
}

// Second pass (one workgroup): the two weighted means.
__global__ __launch_bounds__(64) void env_shift_final(const double2* __restrict__ part, int n0, int n1,
                                                      double* __restrict__ out) {
  if (threadIdx.x >= 2) return;
  const int s = threadIdx.x, b0 = s ? n0 : 0, b1 = s ? n0 + n1 : n0;
  double num = 0.0, den = 0.0;
  for (int b = b0; b < b1; ++b) {
    num += part[b].x;
    den += part[b].y;
  }
  out[s] = (den > 0.0 && isfinite(num)) ? num / den : 0.0;
}

// Second phase of split chains: partial slots summed in slot order (fixed,
// so results stay bit-reproducible), direct terms added, output written.
__global__ __launch_bounds__(256) void reduce_parts(Bufs bufs, double* __restrict__ Cbase,
                                                    const double2* __restrict__ part,
                                                    const DevRed* __restrict__ reds,
                                                    const DevOut* __restrict__ outs,
                                                    const DevTerm* __restrict__ terms) {
  const DevRed rd = reds[blockIdx.x];
  const DevOut ob = outs[rd.out];
  double2* C = reinterpret_cast<double2*>(Cbase) + ob.c_off;
  for (int e = threadIdx.x; e < kSlotDim * kSlotDim; e += 256) {
    const int lr = e % kSlotDim, lc = e / kSlotDim;
    const int row = rd.m0 + lr, col = rd.n0 + lc;
    if (row >= ob.M || col >= ob.N) continue;
    double vr = 0.0, vi = 0.0;
    for (int q = 0; q < rd.nparts; ++q) {
      const double2 v = part[(int64_t)(rd.slot0 + q) * kSlotDim * kSlotDim + e];
      vr += v.x;
      vi += v.y;
    }
    for (int d = ob.d_begin; d < ob.d_end; ++d) {
      const DevTerm dt = terms[d];
      if ((dt.ops & 48) && !bufs.shift) continue;
      const int64_t idx = (dt.ops & 1) ? (int64_t)col + (int64_t)row * dt.lda : (int64_t)row + (int64_t)col * dt.lda;
      const double2 x = (reinterpret_cast<const double2*>(bufs.p[dt.a_buf]) + dt.a_off)[idx];
      double c = dt.coef;
      if (dt.ops & 16) c *= bufs.shift[0];
      if (dt.ops & 32) c *= bufs.shift[1];
      vr += c * x.x;
      vi += (dt.ops & 2) ? -c * x.y : c * x.y;
    }
    if (bufs.bad && !(isfinite(vr) && isfinite(vi))) *bufs.bad = 1;
    C[(int64_t)row + (int64_t)col * ob.ldc] = make_double2(vr, vi);
  }
}

// Two entry kernels with the same body, so that profiles separate the
// effective-Hamiltonian applies from every other grouped GEMM (environment
// updates, gathers, Gram matrices, copies).
template <typename T, int WM, int WN, bool SH>
__global__ __launch_bounds__(64 * WM * WN) void heff_gemm(Bufs bufs, double* __restrict__ C,
                                                         double2* __restrict__ part,
                                                         const DevTile* __restrict__ tiles,
                                                         const DevOut* __restrict__ outs,
                                                         const DevTerm* __restrict__ terms) {
  gemm_body<T, WM, WN, SH>(bufs, C, part, tiles, outs, terms, blockIdx.x);
}
template <typename T, int WM, int WN, bool SH>
__global__ __launch_bounds__(64 * WM * WN) void block_gemm(Bufs bufs, double* __restrict__ C,
                                                          double2* __restrict__ part,
                                                          const DevTile* __restrict__ tiles,
                                                          const DevOut* __restrict__ outs,
                                                          const DevTerm* __restrict__ terms) {
  gemm_body<T, WM, WN, SH>(bufs, C, part, tiles, outs, terms, blockIdx.x);
}

// Persistent form of the effective-Hamiltonian launch: a grid of as many
// workgroups as fit on the device at once takes the (cost-ordered) tiles from
// a device counter, one at a time, until none is left.  Every workgroup ends
// when the counter passes the tile count, so the grid drains by itself.
template <typename T, int WM, int WN, bool SH>
__global__ __launch_bounds__(64 * WM * WN) __attribute__((amdgpu_waves_per_eu(3)))
void heff_gemm_persistent(Bufs bufs, double* __restrict__ C,
                                                                    double2* __restrict__ part,
                                                                    const DevTile* __restrict__ tiles,
                                                                    const DevOut* __restrict__ outs,
                                                                    const DevTerm* __restrict__ terms, int ntiles,
                                                                    int* __restrict__ counter) {
  __shared__ int next;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(counter, 1);
    __syncthreads();
    const int tile = next;
    if (tile >= ntiles) return;
    gemm_body<T, WM, WN, SH>(bufs, C, part, tiles, outs, terms, tile);
    __syncthreads();   // every thread has read `next` before it is overwritten
  }
}

__global__ void reset_counter(int* __restrict__ counter) {
  if (threadIdx.x == 0) *counter = 0;
}

// Workgroups of heff_gemm_persistent<T, 2, 2, SH> resident at once on the device.
template <typename T, bool SH>
int resident_groups(tdvp_ctx* ctx) {
  static int cached[64] = {};
  const int dev = ctx->device < 64 ? ctx->device : 0;
  if (cached[dev]) return cached[dev];
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, heff_gemm_persistent<T, 2, 2, SH>, 256, 0) !=
          hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess ||
      per_cu < 1 || cus < 1)
    return 256;
  return cached[dev] = per_cu * cus;
}

template <typename T, bool SH>
void launch_persistent(tdvp_ctx* ctx, int ntiles, const Bufs& bufs, double* C, double2* part, const DevTile* tiles,
                       const DevArrays& a, int* counter) {
  const int g = std::max(1, std::min(ntiles, resident_groups<T, SH>(ctx)));
  hipLaunchKernelGGL(reset_counter, dim3(1), dim3(64), 0, ctx->stream, counter);
  hipLaunchKernelGGL((heff_gemm_persistent<T, 2, 2, SH>), dim3(g), dim3(256), 0, ctx->stream, bufs, C, part, tiles,
                     a.outs, a.terms, ntiles, counter);
}

template <typename T, int WM, int WN>
void launch_one(tdvp_ctx* ctx, bool heff, int ntiles, const Bufs& bufs, double* C, double2* part,
                const DevTile* tiles, const DevArrays& a) {
  const dim3 g(ntiles), b(64 * WM * WN);
  if (bufs.shift) {
    if (heff)
      hipLaunchKernelGGL((heff_gemm<T, WM, WN, true>), g, b, 0, ctx->stream, bufs, C, part, tiles, a.outs, a.terms);
    else
      hipLaunchKernelGGL((block_gemm<T, WM, WN, true>), g, b, 0, ctx->stream, bufs, C, part, tiles, a.outs, a.terms);
  } else {
    if (heff)
      hipLaunchKernelGGL((heff_gemm<T, WM, WN, false>), g, b, 0, ctx->stream, bufs, C, part, tiles, a.outs, a.terms);
    else
      hipLaunchKernelGGL((block_gemm<T, WM, WN, false>), g, b, 0, ctx->stream, bufs, C, part, tiles, a.outs, a.terms);
  }
}

}  // namespace

hipError_t Allocator::get(void** p, size_t n) const {
  hipError_t e;
  if (!alloc_fn) {
    e = hipMalloc(p, n);
  } else {
    *p = alloc_fn(n, user);
    e = *p ? hipSuccess : hipErrorOutOfMemory;
  }
  if (e == hipSuccess && *p) {
    std::lock_guard<std::mutex> lk(mu);
    held[*p] = n;
    live += n;
    peak = std::max(peak, live);
  }
  return e;
}

void Allocator::put(void* p) const {
  if (!p) return;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = held.find(p);
    if (it != held.end()) {
      live -= it->second;
      held.erase(it);
    }
  }
  if (free_fn) free_fn(p, user);
  else (void)hipFree(p);
}

Program::~Program() {
  for (hipEvent_t e : tune_ev)
    if (e) (void)hipEventDestroy(e);
  if (d_by_out) {
    if (pool && pool->al) pool->al->put(d_by_out);
    else (void)hipFree(d_by_out);
  }
  if (!d_mem) return;
  if (pool) pool->free[cls].push_back(d_mem);
  else (void)hipFree(d_mem);
}

ProgPool::~ProgPool() {
  for (auto& kv : free)
    for (void* p : kv.second) {
      if (al) al->put(p);
      else (void)hipFree(p);
    }
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

// Workgroups go to the eight XCDs (each with its own L2) in round-robin order
// of their index.  Items are grouped by output block (its tiles share operand
// rows and columns), groups are spread over the XCDs by decreasing cost, and
// the per-XCD queues (each still by decreasing cost) are interleaved so that
// index i runs on XCD i mod 8.  TDVP_XCD=0 keeps the plain cost order.
constexpr int kXcds = 8;
constexpr int kCusPerXcd = 32;   // MI355X: 256 compute units in eight XCDs

// Snake order of wave-tile workgroups within each XCD (TDVP_WAVE_SNAKE=0
// keeps the plain cost order; read when a program is built).
static bool wave_snake() {
  static const bool on = [] {
    const char* e = std::getenv("TDVP_WAVE_SNAKE");
    return !(e && std::atoi(e) == 0);
  }();
  return on;
}

template <typename Item>
static std::vector<Item> xcd_order(const std::vector<Item>& items, int per = 1) {
  static const bool on = [] {
    const char* e = std::getenv("TDVP_XCD");
    return !(e && std::atoi(e) == 0);
  }();
  if (!on || items.size() < 2 * (size_t)kXcds * per) return items;
  std::map<int, double> gcost;
  for (const Item& it : items) gcost[it.t.out] += it.cost;
  std::vector<std::pair<double, int>> groups;
  for (auto& kv : gcost) groups.push_back({kv.second, kv.first});
  std::stable_sort(groups.begin(), groups.end(), [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
    return a.first > b.first;
  });
  double load[kXcds] = {};
  std::map<int, int> home;
  for (auto& g : groups) {
    int x = (int)(std::min_element(load, load + kXcds) - load);
    home[g.second] = x;
    load[x] += g.first;
  }
  std::vector<Item> q[kXcds];
  for (const Item& it : items) q[home[it.t.out]].push_back(it);   // stays cost-ordered
  if (per > 1 && wave_snake()) {
    // Wave tiles: all workgroups are resident at once and an XCD's workgroups
    // go to its compute units in turn, so in every other round of one
    // workgroup per compute unit the order is reversed (the unit that took the
    // heaviest group of one round takes the lightest of the next).
    for (auto& v : q) {
      const size_t round = (size_t)kCusPerXcd * per;
      for (size_t r0 = round; r0 < v.size(); r0 += 2 * round) {
        const size_t r1 = std::min(v.size(), r0 + round);
        std::vector<Item> g;   // the round's workgroups (items in runs of `per`), last one first
        g.reserve(r1 - r0);
        for (size_t e = r1; e > r0;) {
          const size_t b = r0 + (e - r0 - 1) / per * per;   // start of the run that ends at e
          g.insert(g.end(), v.begin() + b, v.begin() + e);
          e = b;
        }
        std::copy(g.begin(), g.end(), v.begin() + r0);
      }
    }
  }
  // `per` consecutive items make one workgroup (wave tiles: four), so the
  // queues are interleaved `per` items at a time
  std::vector<Item> out;
  out.reserve(items.size());
  size_t pos[kXcds] = {};
  while (out.size() < items.size()) {
    for (int x = 0; x < kXcds && out.size() < items.size(); ++x)
      for (int r = 0; r < per && out.size() < items.size(); ++r) {
        int src = x;
        if (pos[src] >= q[src].size()) {   // empty queue: borrow from the fullest one
          size_t best = 0;
          for (int y = 0; y < kXcds; ++y)
            if (q[y].size() - pos[y] > best) {
              best = q[y].size() - pos[y];
              src = y;
            }
        }
        out.push_back(q[src][pos[src]++]);
      }
  }
  return out;
}

static double env_double(const char* name, double dflt) {
  const char* e = std::getenv(name);
  return e ? std::atof(e) : dflt;
}

void Program::finalize() {
  tiles.clear();
  reds.clear();
  nslots = 0;
  // operand ranges per buffer (the elements a launch can read through GEMM terms)
  for (int b = 0; b < kMaxBufs; ++b) blo[b] = bhi[b] = 0;
  bool seen[kMaxBufs] = {};
  auto widen = [&](int b, int64_t lo, int64_t hi) {
    if (b < 0 || b >= kMaxBufs) return;
    if (!seen[b]) {
      blo[b] = lo;
      bhi[b] = hi;
      seen[b] = true;
    } else {
      blo[b] = std::min(blo[b], lo);
      bhi[b] = std::max(bhi[b], hi);
    }
  };
  for (const DevOut& ob : outs)
    for (int t = ob.t_begin; t < ob.t_end; ++t) {
      const DevTerm& d = terms[t];
      if (d.K <= 0 || ob.M <= 0 || ob.N <= 0) continue;
      const int64_t ea = (d.ops & 1) ? (int64_t)(d.K - 1) + (int64_t)(ob.M - 1) * d.lda
                                     : (int64_t)(ob.M - 1) + (int64_t)(d.K - 1) * d.lda;
      const int64_t eb = (d.ops & 4) ? (int64_t)(ob.N - 1) + (int64_t)(d.K - 1) * d.ldb
                                     : (int64_t)(d.K - 1) + (int64_t)(ob.N - 1) * d.ldb;
      widen(d.a_buf, d.a_off, d.a_off + ea + 1);
      widen(d.b_buf, d.b_off, d.b_off + eb + 1);
    }
  tile_mode = default_tile_mode();
  const double thr = tile_threshold();
  // Splitting of long K chains, so that no work item runs much longer than
  // alpha x the mean work per resident workgroup (4 per CU of 64x64 tiles on
  // 256 CUs); the pieces are summed by a second, short kernel in a fixed
  // order.  Default: only large effective-Hamiltonian applies (>= 1e11 flops) are
  // split, alpha = 1 and pieces >= 128 deep (measured: +7 % at chi = 16384,
  // 4.5e11 flops; -4 % at chi = 4096, 1.8e10 flops).
  const bool big_apply = role == 1 && flops >= 1e11;
  const double alpha = split_alpha >= 0.0 ? split_alpha : (big_apply ? 1.0 : 0.0);
  const int kmin = split_kmin > 0 ? split_kmin : 128;
  static const int max_slots = (int)env_double("TDVP_SPLIT_MAXSLOTS", 2048);
  struct Item {
    DevTile t;
    double cost;   // issued matrix work, in units of a 64 x 64 x 1 step
    double kc;     // chain depth issued (K, rounded to 4 per step)
    bool big;
  };
  std::vector<Item> items;
  double total = 0.0;
  for (int o = 0; o < (int)outs.size(); ++o) {
    const DevOut& ob = outs[o];
    double kc = 0;
    for (int t = ob.t_begin; t < ob.t_end; ++t) {
      int k0 = 0;
      do {
        kc += (std::min(kHostKStep, terms[t].K - k0) + 3) / 4 * 4;
        k0 += kHostKStep;
      } while (k0 < terms[t].K);
    }
    // 64x64 tiles carry twice the arithmetic intensity of 32x32 ones: prefer
    // them unless their padding costs more than the threshold factor
    bool big = tile_mode == 2 || (tile_mode == 0 && tile_use(ob.M, ob.N, 64) >= thr * tile_use(ob.M, ob.N, 32));
    int tt = big ? 64 : 32;
    for (int m0 = 0; m0 < ob.M; m0 += tt)
      for (int n0 = 0; n0 < ob.N; n0 += tt) {
        double am = (double)((std::min(tt, ob.M - m0) + 15) / 16 * 16);
        double an = (double)((std::min(tt, ob.N - n0) + 15) / 16 * 16);
        Item it;
        it.t = DevTile{o, m0, n0, -1, ob.t_begin, 0, ob.t_end, 0};
        it.kc = kc;
        it.cost = am * an / 4096.0 * (kc + 4.0 * (ob.d_end - ob.d_begin)) + 1.0;
        it.big = big;
        total += it.cost;
        items.push_back(it);
      }
  }
  // chunk cap: alpha x mean work per slot, at least kmin deep; raised until
  // the partial slots fit
  double cap = alpha > 0.0 ? std::max(alpha * total / 1024.0, 1.0) : 1e300;
  std::vector<int> nparts(items.size(), 1);
  for (int tries = 0; tries < 32; ++tries) {
    int ns = 0;
    for (size_t i = 0; i < items.size(); ++i) {
      const Item& it = items[i];
      int n = (int)std::ceil(it.cost / cap);
      n = std::max(1, std::min(n, (int)(it.kc / kmin)));
      nparts[i] = n;
      if (n > 1) ns += n;
    }
    if (ns <= max_slots) break;
    cap *= 1.5;
  }
  std::vector<Item> out64, out32;
  for (size_t i = 0; i < items.size(); ++i) {
    const Item& it = items[i];
    auto& dst = it.big ? out64 : out32;
    const int n = nparts[i];
    if (n == 1) {
      dst.push_back(it);
      continue;
    }
    const DevOut& ob = outs[it.t.out];
    DevRed rd{it.t.out, it.t.m0, it.t.n0, nslots, n, {0, 0, 0}};
    reds.push_back(rd);
    // walk the chain's steps, cutting after the step that reaches q/n of its depth
    double acc = 0.0;
    int q = 0;
    Item piece = it;
    piece.t.t0 = ob.t_begin;
    piece.t.k0 = 0;
    double piece_kc = 0.0;
    for (int t = ob.t_begin; t < ob.t_end; ++t) {
      int k0 = 0;
      do {
        double d = (std::min(kHostKStep, terms[t].K - k0) + 3) / 4 * 4;
        acc += d;
        piece_kc += d;
        int tn = t, kn = k0 + kHostKStep;
        if (kn >= terms[t].K) { kn = 0; ++tn; }
        const bool last = tn == ob.t_end;
        if (q < n - 1 && !last && acc >= it.kc * (q + 1) / n) {
          piece.t.t1 = tn;
          piece.t.k1 = kn;
          piece.t.slot = nslots + q;
          piece.cost = it.cost * piece_kc / std::max(it.kc, 1.0);
          dst.push_back(piece);
          ++q;
          piece.t.t0 = tn;
          piece.t.k0 = kn;
          piece_kc = 0.0;
        }
        k0 += kHostKStep;
      } while (k0 < terms[t].K);
    }
    piece.t.t1 = ob.t_end;
    piece.t.k1 = 0;
    piece.t.slot = nslots + q;
    piece.cost = it.cost * piece_kc / std::max(it.kc, 1.0);
    dst.push_back(piece);
    reds.back().nparts = q + 1;
    nslots += q + 1;
  }
  auto bycost = [](const Item& a, const Item& b) { return a.cost > b.cost; };
  std::stable_sort(out64.begin(), out64.end(), bycost);
  std::stable_sort(out32.begin(), out32.end(), bycost);
  n64 = (int)out64.size();
  for (const Item& it : xcd_order(out64)) tiles.push_back(it.t);
  for (const Item& it : xcd_order(out32)) tiles.push_back(it.t);
  // autotuning candidates for effective-Hamiltonian programs without split chains
  alt.clear();
  static const bool autotune = [] {
    const char* e = std::getenv("TDVP_AUTOTUNE");
    return !(e && std::atoi(e) == 0);
  }();
  if (autotune && role == 1 && nslots == 0) {
    Tiling a0;
    a0.tiles = tiles;
    a0.n64 = n64;
    a0.mode = tile_mode;
    alt.push_back(a0);
    for (int mode : {1, 0, 2})
      if (mode != tile_mode) {
        Tiling a;
        tile_only(mode, a);
        alt.push_back(a);
      }
    // the all-64x64 tiles once more, launched as a persistent grid, and the
    // all-32x32 tiles as wave tiles
    const size_t nbase = alt.size();
    for (size_t v = 0; v < nbase; ++v) {
      if (alt[v].mode == 2) {
        Tiling a = alt[v];
        a.mode = 3;
        a.persistent = true;
        alt.push_back(a);
      }
      if (alt[v].mode == 1) {
        Tiling a;
        tile_only(1, a, 4);
        a.mode = 4;
        a.wave = true;
        alt.push_back(a);
      }
    }
  }
}

void Program::tile_only(int mode, Tiling& out, int per) const {
  struct It {
    DevTile t;
    double cost;
  };
  std::vector<It> t64, t32;
  const double thr = tile_threshold();
  for (int o = 0; o < (int)outs.size(); ++o) {
    const DevOut& ob = outs[o];
    double kc = 0;
    for (int t = ob.t_begin; t < ob.t_end; ++t) kc += (terms[t].K + 3) / 4 * 4;
    bool big = mode == 2 || (mode == 0 && tile_use(ob.M, ob.N, 64) >= thr * tile_use(ob.M, ob.N, 32));
    int tt = big ? 64 : 32;
    for (int m0 = 0; m0 < ob.M; m0 += tt)
      for (int n0 = 0; n0 < ob.N; n0 += tt) {
        double am = (double)((std::min(tt, ob.M - m0) + 15) / 16 * 16);
        double an = (double)((std::min(tt, ob.N - n0) + 15) / 16 * 16);
        It it{DevTile{o, m0, n0, -1, ob.t_begin, 0, ob.t_end, 0}, am * an * (kc + 4.0 * (ob.d_end - ob.d_begin)) + 1.0};
        (big ? t64 : t32).push_back(it);
      }
  }
  auto bycost = [](const It& a, const It& b) { return a.cost > b.cost; };
  std::stable_sort(t64.begin(), t64.end(), bycost);
  std::stable_sort(t32.begin(), t32.end(), bycost);
  out.tiles.clear();
  out.n64 = (int)t64.size();
  out.mode = mode;
  for (const It& it : xcd_order(t64, per)) out.tiles.push_back(it.t);
  for (const It& it : xcd_order(t32, per)) out.tiles.push_back(it.t);
}

DeviceBuffer::~DeviceBuffer() { release(); }

void DeviceBuffer::release() {
  if (p) {
    if (al) al->put(p);
    else (void)hipFree(p);
  }
  p = nullptr;
  bytes = 0;
}

hipError_t DeviceBuffer::ensure(size_t n) {
  if (n <= bytes) return hipSuccess;
  release();
  size_t want = std::max(n, (size_t)256);
  hipError_t e = al ? al->get(&p, want) : hipMalloc(&p, want);
  if (e == hipSuccess) bytes = want;
  else p = nullptr;
  return e;
}

int bad_flag(tdvp_ctx* ctx, int** flag) {
  *flag = nullptr;
  if (ctx->ws_flag.p) {
    *flag = (int*)ctx->ws_flag.p;
    return TDVP_OK;
  }
  TDVP_HIP(ctx, ctx->ws_flag.ensure(256));
  TDVP_HIP(ctx, hipMemsetAsync(ctx->ws_flag.p, 0, 256, ctx->stream));
  *flag = (int*)ctx->ws_flag.p;
  return TDVP_OK;
}

int upload(tdvp_ctx* ctx, Program& p) {
  size_t bt = p.terms.size() * sizeof(DevTerm), bo = p.outs.size() * sizeof(DevOut),
         bl = p.tiles.size() * sizeof(DevTile), br = p.reds.size() * sizeof(DevRed),
         bs = p.shift_meta.size() * sizeof(int64_t);
  size_t total = bt + bo + bl + br + bs + 5 * 256;
  for (auto& a : p.alt) total += a.tiles.size() * sizeof(DevTile) + 256;
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
    TDVP_HIP(ctx, ctx->alloc->get(&p.d_mem, cls));
  }
  char* base = (char*)p.d_mem;
  auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
  p.d_terms = (DevTerm*)base;
  p.d_outs = (DevOut*)(base + align(bt));
  p.d_tiles = (DevTile*)(base + align(bt) + align(bo));
  p.d_reds = (DevRed*)(base + align(bt) + align(bo) + align(bl));
  p.d_shift_meta = (int64_t*)(base + align(bt) + align(bo) + align(bl) + align(br));
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
  if (br) std::memcpy(h + align(bt) + align(bo) + align(bl), p.reds.data(), br);
  if (bs) std::memcpy(h + align(bt) + align(bo) + align(bl) + align(br), p.shift_meta.data(), bs);
  size_t used = align(bt) + align(bo) + align(bl) + align(br) + align(bs);
  for (auto& a : p.alt) {
    const size_t ba = a.tiles.size() * sizeof(DevTile);
    a.d_tiles = (DevTile*)(base + used);
    if (ba) std::memcpy(h + used, a.tiles.data(), ba);
    used += align(ba);
  }
  TDVP_HIP(ctx, hipMemcpyAsync(p.d_mem, h, used, hipMemcpyHostToDevice, ctx->stream));
  if (!ctx->upload_done) TDVP_HIP(ctx, hipEventCreateWithFlags(&ctx->upload_done, hipEventDisableTiming));
  TDVP_HIP(ctx, hipEventRecord(ctx->upload_done, ctx->stream));
  return TDVP_OK;
}

std::shared_ptr<Program> cache_get(ProgCache& c, uint64_t key, const std::vector<uint64_t>& sig) {
  for (auto it = c.begin(); it != c.end(); ++it)
    if (it->first == key && it->second->sig == sig) {
      auto p = it->second;
      c.splice(c.begin(), c, it);
      return p;
    }
  return nullptr;
}

void cache_put(ProgCache& c, uint64_t key, std::shared_ptr<Program> p) {
  c.emplace_front(key, std::move(p));
  while (c.size() > 24) c.pop_back();
}

std::shared_ptr<Program> cache_get(tdvp_ctx* ctx, uint64_t key, const std::vector<uint64_t>& sig) {
  return cache_get(ctx->cache, key, sig);
}

void cache_put(tdvp_ctx* ctx, uint64_t key, std::shared_ptr<Program> p) { cache_put(ctx->cache, key, std::move(p)); }

static int launch_core(tdvp_ctx* ctx, const Program& p, const DevArrays& a, int ntiles, int n64,
                       const DevTile* d_tiles, const Bufs& bufs, double* C, int precision, const LaunchWs* ws,
                       bool persistent = false, bool wave = false);
static DevArrays arrays_of(const Program& p) { return DevArrays{p.d_terms, p.d_outs, p.d_reds, p.d_shift_meta}; }

// Autotuner step: which tiling this launch uses, with its events.  Every
// candidate is launched kTuneRounds times, each bracketed by events; at the
// first launch after the last measurement (the caller has synchronised in
// between, as the Krylov loop does every iteration; otherwise this waits) the
// fastest total wins.  The decision is kept in the context by program class
// (role, half-octave of flops): later programs of that class, such as the
// next bonds of a sweep, take it without measuring.
static int tune_class(const Program& p) {
  return p.role * 1000 + (int)std::floor(2.0 * std::log2(std::max(p.flops, 1.0)));
}

static int tune_pick(tdvp_ctx* ctx, const Program& p, hipEvent_t*& ev0, hipEvent_t*& ev1) {
  ev0 = ev1 = nullptr;
  const int nv = (int)p.alt.size();
  if (nv <= 1) return -1;
  if (p.tuned >= 0) return p.tuned;
  if (p.tune_next == 0) {   // a class already decided in this context: take its choice
    auto it = ctx->tuned_modes.find(tune_class(p));
    if (it != ctx->tuned_modes.end())
      for (int v = 0; v < nv; ++v)
        if (p.alt[v].mode == it->second) return p.tuned = v;
  }
  const int need = nv * Program::kTuneRounds;
  if (p.tune_next < need) {
    if (p.tune_ev.empty()) {
      p.tune_ev.assign(2 * need, nullptr);
      for (auto& e : p.tune_ev)
        if (hipEventCreate(&e) != hipSuccess) {
          e = nullptr;
          p.tuned = 0;
          return 0;
        }
    }
    const int k = p.tune_next++;
    ev0 = &p.tune_ev[2 * k];
    ev1 = &p.tune_ev[2 * k + 1];
    return k % nv;
  }
  std::vector<float> tot(nv, 0.0f);
  for (int k = 0; k < need; ++k) {
    float ms = 0.0f;
    if (hipEventSynchronize(p.tune_ev[2 * k + 1]) != hipSuccess ||
        hipEventElapsedTime(&ms, p.tune_ev[2 * k], p.tune_ev[2 * k + 1]) != hipSuccess) {
      ms = 1e30f;
      (void)hipGetLastError();   // a failed timing query ranks the candidate last; it is no launch error
    }
    tot[k % nv] += ms;
  }
  p.tuned = (int)(std::min_element(tot.begin(), tot.end()) - tot.begin());
  ctx->tuned_modes[tune_class(p)] = p.alt[p.tuned].mode;
  if (ctx->verbose >= 2) {
    std::string msg;
    for (int v = 0; v < nv; ++v) msg += " mode" + std::to_string(p.alt[v].mode) + "=" + std::to_string(tot[v]);
    std::fprintf(stderr, "[tdvp]   autotune:%s ms -> mode %d\n", msg.c_str(), p.alt[p.tuned].mode);
  }
  return p.tuned;
}

// Baseline schedule: one launch per output block (64x64 tiles of that block),
// selected with TDVP_PER_BLOCK=1 at launch time; same work, same results.
static int launch_per_block(tdvp_ctx* ctx, const Program& p, const Bufs& bufs, double* C, int precision) {
  if (p.blk_begin.empty()) {
    Program::Tiling t64;
    p.tile_only(2, t64);
    std::vector<DevTile> v = t64.tiles;
    std::stable_sort(v.begin(), v.end(), [](const DevTile& a, const DevTile& b) { return a.out < b.out; });
    p.blk_begin.push_back(0);
    for (size_t i = 1; i <= v.size(); ++i)
      if (i == v.size() || v[i].out != v[i - 1].out) p.blk_begin.push_back((int)i);
    TDVP_HIP(ctx, ctx->alloc->get(&p.d_by_out, sizeof(DevTile) * std::max<size_t>(v.size(), 1)));
    TDVP_HIP(ctx, hipMemcpy(p.d_by_out, v.data(), sizeof(DevTile) * v.size(), hipMemcpyHostToDevice));
  }
  const DevTile* base = (const DevTile*)p.d_by_out;
  for (size_t b = 0; b + 1 < p.blk_begin.size(); ++b) {
    const int n = p.blk_begin[b + 1] - p.blk_begin[b];
    int rc = launch_core(ctx, p, arrays_of(p), n, n, base + p.blk_begin[b], bufs, C, precision, nullptr);
    if (rc) return rc;
  }
  return TDVP_OK;
}

int launch_gemm(tdvp_ctx* ctx, const Program& p, const Bufs& bufs, double* C, int precision) {
  if (p.tiles.empty()) return TDVP_OK;
  if (p.nslots == 0) {
    const char* e = std::getenv("TDVP_PER_BLOCK");
    if (e && std::atoi(e) == 1) return launch_per_block(ctx, p, bufs, C, precision);
  }
  // FP64 launches only: there every tiling gives identical results, while the
  // reduced-precision kernels differ between 64x64 and 32x32 tiles
  hipEvent_t *ev0 = nullptr, *ev1 = nullptr;
  int v = -1;
  // measurement and test hook, read at every launch: TDVP_FORCE_TILING=m runs
  // the candidate of mode m (0-2 tilings, 3 the persistent launch, 4 wave
  // tiles) instead, and the autotuner is left alone
  if (const char* f = std::getenv("TDVP_FORCE_TILING")) {
    const int m = std::atoi(f);
    for (int c = 0; c < (int)p.alt.size(); ++c)
      if (p.alt[c].mode == m && (precision == TDVP_FP64 || !p.alt[c].persistent) &&
          (precision != TDVP_BF16X3 || !p.alt[c].wave))
        v = c;
  }
  if (v < 0 && precision == TDVP_FP64) v = tune_pick(ctx, p, ev0, ev1);
  if (v >= 0) {   // the chosen (or measured) tiling replaces the active one
    const Program::Tiling& a = p.alt[v];
    if (ev0) TDVP_HIP(ctx, hipEventRecord(*ev0, ctx->stream));
    int rc = launch_core(ctx, p, arrays_of(p), (int)a.tiles.size(), a.n64, a.d_tiles, bufs, C, precision, nullptr,
                         a.persistent, a.wave);
    if (ev1) TDVP_HIP(ctx, hipEventRecord(*ev1, ctx->stream));
    return rc;
  }
  return launch_core(ctx, p, arrays_of(p), (int)p.tiles.size(), p.n64, p.d_tiles, bufs, C, precision, nullptr);
}

int launch_gemm_tiles(tdvp_ctx* ctx, const Program& p, const Bufs& bufs, double* C, int precision) {
  return launch_core(ctx, p, arrays_of(p), (int)p.tiles.size(), p.n64, p.d_tiles, bufs, C, precision, nullptr);
}

int launch_gemm_ws(tdvp_ctx* ctx, const Program& p, const DevArrays& a, const DevTile* d_tiles, const Bufs& bufs,
                   double* C, int precision, const LaunchWs& ws) {
  return launch_core(ctx, p, a, (int)p.tiles.size(), p.n64, d_tiles, bufs, C, precision, &ws);
}

size_t partial_slot_bytes(int nslots) { return sizeof(double2) * (size_t)nslots * kSlotDim * kSlotDim; }

// ws == nullptr: partial slots and shifts live in the context's grow-only
// workspaces; otherwise in the caller's (ws->part, ws->shift), which are
// large enough (checked by the caller).
static int launch_core(tdvp_ctx* ctx, const Program& p, const DevArrays& arr, int ntiles, int n64,
                       const DevTile* d_tiles, const Bufs& bufs, double* C, int precision, const LaunchWs* ws,
                       bool persistent, bool wave) {
  if (ntiles == 0) return TDVP_OK;
  double2* part = nullptr;
  if (p.nslots > 0) {
    if (ws) {
      part = ws->part;
    } else {
      TDVP_HIP(ctx, ctx->ws_part.ensure(partial_slot_bytes(p.nslots)));
      part = (double2*)ctx->ws_part.p;
    }
  }
  if (precision == TDVP_BF16X3 && ntiles > n64) {
    // the split-BF16 kernel exists for 64x64 tiles only: take the program's
    // all-64x64 tiling, or refuse rather than run FP32 under the BF16X3 label
    const Program::Tiling* t64 = nullptr;
    for (const auto& a : p.alt)
      if (a.mode == 2) t64 = &a;
    if (ws || !t64 || !t64->d_tiles)
      return set_error(ctx, TDVP_E_INVALID, "split-BF16 products need 64x64 tiles (tile mode 2)");
    ntiles = (int)t64->tiles.size();
    n64 = t64->n64;
    d_tiles = t64->d_tiles;
  }
  const int n32 = ntiles - n64;
  const DevTile* t32 = d_tiles + n64;
  const bool heff = p.role == 1;
  Bufs bf = bufs;
  bf.shift = nullptr;
  if (int rc = bad_flag(ctx, &bf.bad)) return rc;
  Slices sl{};
  uint4* slice_base = nullptr;
  if (precision == TDVP_BF16X3 && n64 > 0) {
    if (ws) return set_error(ctx, TDVP_E_INVALID, "split-BF16 products need the context's operand-slice workspace");
    size_t nrec = 0;
    for (int b = 0; b < kMaxBufs; ++b) nrec += (size_t)(p.bhi[b] - p.blo[b]);
    TDVP_HIP(ctx, ctx->ws_slices.ensure(sizeof(uint4) * std::max<size_t>(nrec, 1)));
    slice_base = (uint4*)ctx->ws_slices.p;
    size_t cur = 0;
    for (int b = 0; b < kMaxBufs; ++b) {
      if (p.bhi[b] <= p.blo[b]) continue;
      sl.p[b] = slice_base + cur;
      sl.lo[b] = p.blo[b];
      cur += (size_t)(p.bhi[b] - p.blo[b]);
    }
  }
  if (precision != TDVP_FP64 && p.nshift[0] + p.nshift[1] > 0) {
    const int nb = p.nshift[0] + p.nshift[1];
    double* out;
    if (ws) {
      out = ws->shift;
    } else {
      TDVP_HIP(ctx, ctx->ws_shift.ensure(shift_bytes(nb)));
      out = (double*)ctx->ws_shift.p;
    }
    double2* partial = (double2*)out + 1;
    hipLaunchKernelGGL(env_shift_parts, dim3(nb), dim3(256), 0, ctx->stream, bufs, arr.shift_meta,
                       p.nshift[0], partial);
    hipLaunchKernelGGL(env_shift_final, dim3(1), dim3(64), 0, ctx->stream, (const double2*)partial, p.nshift[0],
                       p.nshift[1], out);
    bf.shift = out;
  }
  if (slice_base) {   // operand records, once per buffer; shifted diagonals re-made from E - shift
    for (int b = 0; b < kMaxBufs; ++b) {
      if (!sl.p[b]) continue;
      const int64_t n = p.bhi[b] - p.blo[b];
      const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
      hipLaunchKernelGGL(slice_records, dim3(g), dim3(256), 0, ctx->stream,
                         reinterpret_cast<const double2*>(bufs.p[b]) + p.blo[b], const_cast<uint4*>(sl.p[b]), n);
    }
    for (int s = 0; s < 2 && bf.shift; ++s) {
      const int b = 1 + s;
      const int nb = p.nshift[s];
      if (nb == 0 || !sl.p[b]) continue;
      hipLaunchKernelGGL(slice_fix_diag, dim3(nb), dim3(256), 0, ctx->stream,
                         reinterpret_cast<const double2*>(bufs.p[b]), const_cast<uint4*>(sl.p[b]), p.blo[b], p.bhi[b],
                         arr.shift_meta + 3 * (s ? p.nshift[0] : 0), (const double*)bf.shift + s);
    }
  }
  if (n64 > 0) {
    if (precision == TDVP_BF16X3) {
      const dim3 g(n64), bl(256);
      if (bf.shift) {
        if (heff) hipLaunchKernelGGL((heff_gemm_b3<true>), g, bl, 0, ctx->stream, bf, sl, C, part, d_tiles, arr.outs, arr.terms);
        else hipLaunchKernelGGL((block_gemm_b3<true>), g, bl, 0, ctx->stream, bf, sl, C, part, d_tiles, arr.outs, arr.terms);
      } else {
        if (heff) hipLaunchKernelGGL((heff_gemm_b3<false>), g, bl, 0, ctx->stream, bf, sl, C, part, d_tiles, arr.outs, arr.terms);
        else hipLaunchKernelGGL((block_gemm_b3<false>), g, bl, 0, ctx->stream, bf, sl, C, part, d_tiles, arr.outs, arr.terms);
      }
    } else if (precision == TDVP_FP32) {
      launch_one<float, 2, 2>(ctx, heff, n64, bf, C, part, d_tiles, arr);
    } else if (persistent && heff && !ws) {
      // the work counter sits in the context's flag buffer, after the non-finite flag
      int* counter = (int*)ctx->ws_flag.p + 16;
      if (bf.shift) launch_persistent<double, true>(ctx, n64, bf, C, part, d_tiles, arr, counter);
      else launch_persistent<double, false>(ctx, n64, bf, C, part, d_tiles, arr, counter);
    } else {
      launch_one<double, 2, 2>(ctx, heff, n64, bf, C, part, d_tiles, arr);
    }
  }
  if (n32 > 0) {   // 32x32 tiles (optional tile modes; never under BF16X3, see above)
    if (precision != TDVP_FP64 && wave && heff && p.nslots == 0) {   // FP32 wave tiles
      const dim3 g((unsigned)((n32 + 3) / 4)), b(256);
      if (bf.shift) hipLaunchKernelGGL((heff_gemm_wave<float, true>), g, b, 0, ctx->stream, bf, C, t32, n32, arr.outs, arr.terms);
      else hipLaunchKernelGGL((heff_gemm_wave<float, false>), g, b, 0, ctx->stream, bf, C, t32, n32, arr.outs, arr.terms);
    } else if (precision != TDVP_FP64) {
      launch_one<float, 1, 1>(ctx, heff, n32, bf, C, part, t32, arr);
    } else if (wave && heff && p.nslots == 0) {   // four wave tiles per workgroup
      hipLaunchKernelGGL((heff_gemm_wave<double, false>), dim3((unsigned)((n32 + 3) / 4)), dim3(256), 0, ctx->stream,
                         bf, C, t32, n32, arr.outs, arr.terms);
    } else {
      launch_one<double, 1, 1>(ctx, heff, n32, bf, C, part, t32, arr);
    }
  }
  if (!p.reds.empty())
    hipLaunchKernelGGL(reduce_parts, dim3((unsigned)p.reds.size()), dim3(256), 0, ctx->stream, bf, C,
                       (const double2*)part, arr.reds, arr.outs, arr.terms);
  TDVP_HIP(ctx, hipGetLastError());
  return TDVP_OK;
}

}  // namespace tdvp

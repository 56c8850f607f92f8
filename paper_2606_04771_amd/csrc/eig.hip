// Batched Hermitian eigensolver pieces for the two-site split (supplementary
// section S2.2: the SVD of each symmetry sector's two-site matrix, done here
// through the eigendecomposition of its Gram matrix).
//
// Hermitian matrices (column-major, full storage, each n x n with its own
// leading dimension) are reduced to real symmetric tridiagonal form
// T = Q^H A Q by Householder reflectors Q = H_0 H_1 ... H_{n-2},
// H_k = I - tau_k v_k v_k^H (the reduction of Golub and Van Loan, section
// 8.3.1, in LAPACK's complex convention: beta = e_k real, v_k(k+1) = 1).
// Column k of every matrix of a set (all the large Gram matrices of one
// split, of different sizes) is ONE launch: every workgroup of a matrix
// recomputes the column's reflector from the previous column's rank-2 update
// (O(n) redundant work), then applies that update to its own rows of the
// trailing matrix and forms its rows of y_k = tau_k A v_k in the same pass.
// A library solver launches about ten small dependent kernels per column for
// the same reduction.
//
// The tridiagonal eigenproblem is left to a library tridiagonal solver; the
// eigenvectors of A are then Q Z, applied by one launch: one wave per output
// column keeps that column in registers and runs through the reflectors.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.hpp"
#include "ctx.hpp"
#include "eig.hpp"

namespace tdvp {

namespace {

constexpr int kTrdThreads = 256;
constexpr int kTrdRows = 8;   // rows of the trailing matrix per workgroup

__device__ __forceinline__ double wave_total(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;   // every lane holds the sum
}

// Sum of (a, b) over the workgroup, returned to every thread.  `red` holds
// 2 * (threads / 64) doubles; the order of the additions is fixed.
__device__ __forceinline__ double2 group_total(double a, double b, double* red) {
  a = wave_total(a);
  b = wave_total(b);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    red[2 * w] = a;
    red[2 * w + 1] = b;
  }
  __syncthreads();
  double x = 0.0, y = 0.0;
#pragma unroll
  for (int i = 0; i < kTrdThreads / 64; ++i) {
    x += red[2 * i];
    y += red[2 * i + 1];
  }
  __syncthreads();   // `red` may be reused right after
  return make_double2(x, y);
}

// Column k of the reduction for matrix `mat_` of a job (RB rows of its
// trailing matrix per workgroup: block rb_ holds rows k + 1 + RB rb_ ...).
//   A    the matrices (leading dimension lda, lda^2 apart); on entry to
//        launch k the trailing block [k, n)^2 holds
//        A_k + v_{k-1} w_{k-1}^H + w_{k-1} v_{k-1}^H (the last rank-2 update
//        not yet applied), rows/columns < k are no longer read
//   V    reflector store: column k receives v_k on rows [k+1, n)
//   Y    two n-vectors per matrix: y_{k-1} = tau_{k-1} A_{k-1} v_{k-1} is read
//        from slot (k+1)&1, y_k written to slot k&1
//   tau  tau_k (complex), d / e: diagonal / off-diagonal of T (real)
// Launch k writes only columns > k of A, rows it owns, so the column every
// workgroup reads (k) is never written in the same launch.
template <int RB, int S>
__device__ __forceinline__ void trd_column(double2* __restrict__ A, double2* __restrict__ V, double2* __restrict__ Y,
                                           double2* __restrict__ tau, double* __restrict__ dg,
                                           double* __restrict__ eg, const int n, const int lda, const int k,
                                           const int mat_, const int rb_, double2* lds, double* red,
                                           double2* part) {
  double2* vp = lds;           // v_{k-1} on rows [k, n)
  double2* wp = lds + n;       // w_{k-1} on rows [k, n)
  double2* vc = lds + 2 * n;   // column k on rows [k, n), then v_k on rows [k+1, n)
  // S: rows of [k, n) per thread (n <= 256 S)
  const int tid = threadIdx.x;
  const int64_t mat = mat_, nn = (int64_t)n * n;
  double2* Am = A + mat * lda * (int64_t)lda;
  double2* Vm = V + mat * nn;
  const double2* yprev = Y + (2 * mat + ((k + 1) & 1)) * n;
  double2* ynext = Y + (2 * mat + (k & 1)) * n;
  double2* taum = tau + mat * n;
  // own part of the trailing update: row `rown`, columns k + 1 + cg + NCG u
  constexpr int NCG = kTrdThreads / RB, U = 8;
  const int rr = tid % RB, cg = tid / RB;
  const int rown = k + 1 + rb_ * RB + rr;

  // one pass of loads: v_{k-1}, y_{k-1} and column k, rows k + tid + 256 j
  double2 vv[S], ww[S], cc[S];
  double sr = 0.0, si = 0.0;
#pragma unroll
  for (int j = 0; j < S; ++j) {
    const int r = k + tid + j * kTrdThreads;
    vv[j] = ww[j] = cc[j] = make_double2(0.0, 0.0);
    if (r < n) {
      cc[j] = Am[r + (int64_t)k * lda];
      if (k > 0) {
        vv[j] = Vm[r + (int64_t)(k - 1) * n];
        ww[j] = yprev[r];
      }
    }
    sr += ww[j].x * vv[j].x + ww[j].y * vv[j].y;
    si += ww[j].x * vv[j].y - ww[j].y * vv[j].x;
  }
  if (k > 0) {
    // w_{k-1} = y_{k-1} + alpha v_{k-1},  alpha = -(tau_{k-1} / 2) y_{k-1}^H v_{k-1}
    const double2 s = group_total(sr, si, red);
    const double2 t = taum[k - 1];
    const double ar = -0.5 * (t.x * s.x - t.y * s.y), ai = -0.5 * (t.x * s.y + t.y * s.x);
#pragma unroll
    for (int j = 0; j < S; ++j) {
      const int r = k + tid + j * kTrdThreads;
      ww[j] = make_double2(ww[j].x + ar * vv[j].x - ai * vv[j].y, ww[j].y + ar * vv[j].y + ai * vv[j].x);
      if (r < n) {
        vp[r] = vv[j];
        wp[r] = ww[j];
      }
    }
    __syncthreads();
    // column k with the last update applied
    const double2 wk = wp[k], vk = vp[k];
#pragma unroll
    for (int j = 0; j < S; ++j) {
      const double2 v = vv[j], w = ww[j];
      cc[j].x -= (v.x * wk.x + v.y * wk.y) + (w.x * vk.x + w.y * vk.y);
      cc[j].y -= (v.y * wk.x - v.x * wk.y) + (w.y * vk.x - w.x * vk.y);
    }
  }
  double xr = 0.0;
#pragma unroll
  for (int j = 0; j < S; ++j) {
    const int r = k + tid + j * kTrdThreads;
    if (r < n) {
      vc[r] = cc[j];
      if (r >= k + 2) xr += cc[j].x * cc[j].x + cc[j].y * cc[j].y;
    }
  }
  if (rb_ == 0 && tid == 0) dg[mat * n + k] = cc[0].x;
  if (k == n - 1) return;
  // reflector of (alpha, x) = column k below the diagonal
  const double xn2 = group_total(xr, 0.0, red).x;   // its barrier also publishes vc
  const double2 a0 = vc[k + 1];
  double2 t = make_double2(0.0, 0.0), sc = t;
  double beta = a0.x;
  if (xn2 != 0.0 || a0.y != 0.0) {
    beta = -copysign(sqrt(a0.x * a0.x + a0.y * a0.y + xn2), a0.x);
    t = make_double2((beta - a0.x) / beta, -a0.y / beta);
    const double dr = a0.x - beta, di = a0.y, den = dr * dr + di * di;
    sc = make_double2(dr / den, -di / den);   // 1 / (alpha - beta)
  }
  __syncthreads();   // every thread has read alpha before v_k overwrites it
#pragma unroll
  for (int j = 0; j < S; ++j) {
    const int r = k + tid + j * kTrdThreads;
    if (r == k + 1) vc[r] = make_double2(1.0, 0.0);
    else if (r > k + 1 && r < n)
      vc[r] = make_double2(cc[j].x * sc.x - cc[j].y * sc.y, cc[j].x * sc.y + cc[j].y * sc.x);
  }
  if (rb_ == 0 && tid == 0) {
    taum[k] = t;
    eg[mat * n + k] = beta;
  }
  __syncthreads();
  // own rows: apply the last update to columns [k+1, n) and form y_k = tau_k A_{k+1} v_k;
  // U columns per batch with their loads in flight together
  double accr = 0.0, acci = 0.0;
  if (rown < n) {
    double2 vr = make_double2(0.0, 0.0), wr = vr;
    if (k > 0) {
      vr = vp[rown];
      wr = wp[rown];
    }
    auto apply = [&](double2 a, int c) {
      if (k > 0) {
        const double2 vq = vp[c], wq = wp[c];
        a.x -= (vr.x * wq.x + vr.y * wq.y) + (wr.x * vq.x + wr.y * vq.y);
        a.y -= (vr.y * wq.x - vr.x * wq.y) + (wr.y * vq.x - wr.x * vq.y);
        Am[rown + (int64_t)c * lda] = a;
      }
      const double2 x = vc[c];
      accr += a.x * x.x - a.y * x.y;
      acci += a.x * x.y + a.y * x.x;
    };
    for (int c0 = k + 1 + cg; c0 < n; c0 += NCG * U) {
      double2 a[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = c0 + u * NCG;
        a[u] = c < n ? Am[rown + (int64_t)c * lda] : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = c0 + u * NCG;
        if (c < n) apply(a[u], c);
      }
    }
    if (cg == 0) Vm[rown + (int64_t)k * n] = vc[rown];
  }
  part[tid] = make_double2(accr, acci);
  __syncthreads();
  if (cg == 0 && rown < n) {
    double pr = 0.0, pi = 0.0;
    for (int g = 0; g < NCG; ++g) {
      pr += part[g * RB + rr].x;
      pi += part[g * RB + rr].y;
    }
    ynext[rown] = make_double2(t.x * pr - t.y * pi, t.x * pi + t.y * pr);
  }
}

// One launch: column k of every job of the set with n > k.  The workgroups
// are numbered job by job, matrix by matrix, row block by row block.
template <int S>
__global__ __launch_bounds__(kTrdThreads) void k_trd_multi(const TrdJob* __restrict__ jobs, int njobs, int k) {
  extern __shared__ double2 lds[];
  __shared__ double red[2 * (kTrdThreads / 64)];
  __shared__ double2 part[kTrdThreads];
  int blk = (int)blockIdx.x;
  for (int j = 0; j < njobs; ++j) {
    const TrdJob jb = jobs[j];
    if (k >= jb.n) continue;
    const int nrb = max(1, (jb.n - k - 1 + kTrdRows - 1) / kTrdRows);
    if (blk < nrb * jb.count) {
      trd_column<kTrdRows, S>((double2*)jb.A, (double2*)jb.V, (double2*)jb.Y, (double2*)jb.tau, jb.d, jb.e, jb.n,
                           jb.lda, k, blk / nrb, blk % nrb, lds, red, part);
      return;
    }
    blk -= nrb * jb.count;
  }
}

// Eigenvectors of A from those of T: columns c >= c0 of Q Zt, Zt real, one
// wave per column (four per workgroup), n <= 64 * NR.  H_{n-2} is applied
// first; the next reflector is loaded while the current one is applied.
template <int NR>
__global__ __launch_bounds__(kTrdThreads) void k_trd_back(const double* __restrict__ Zt,
                                                           const double2* __restrict__ V,
                                                           const double2* __restrict__ tau, double2* __restrict__ G,
                                                           int n, int c0, int ld) {
  const int lane = threadIdx.x & 63;
  const int c = c0 + (int)blockIdx.x * (kTrdThreads / 64) + (int)(threadIdx.x >> 6);
  if (c >= n) return;   // whole wave; no workgroup barrier below
  const int64_t nn = (int64_t)n * n, mo = (int64_t)blockIdx.y * nn;
  const double2* Vm = V + mo;
  const double2* tm = tau + (int64_t)blockIdx.y * n;
  double zr[NR], zi[NR], nr_[NR], ni_[NR];
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    const int r = lane + 64 * j;
    zr[j] = r < n ? Zt[mo + r + (int64_t)c * n] : 0.0;
    zi[j] = 0.0;
    nr_[j] = ni_[j] = 0.0;
  }
  auto load_v = [&](int k) {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
      const int r = lane + 64 * j;
      double2 v = make_double2(0.0, 0.0);
      if (r > k && r < n) v = Vm[r + (int64_t)k * n];
      nr_[j] = v.x;
      ni_[j] = v.y;
    }
  };
  if (n >= 2) load_v(n - 2);
  for (int k = n - 2; k >= 0; --k) {
    double vr[NR], vi[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
      vr[j] = nr_[j];
      vi[j] = ni_[j];
    }
    const double2 t = tm[k];
    if (k > 0) load_v(k - 1);
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int j = 0; j < NR; ++j) {
      sr += vr[j] * zr[j] + vi[j] * zi[j];
      si += vr[j] * zi[j] - vi[j] * zr[j];
    }
    sr = wave_total(sr);
    si = wave_total(si);
    const double qr = t.x * sr - t.y * si, qi = t.x * si + t.y * sr;   // tau (v^H z)
#pragma unroll
    for (int j = 0; j < NR; ++j) {
      zr[j] -= vr[j] * qr - vi[j] * qi;
      zi[j] -= vr[j] * qi + vi[j] * qr;
    }
  }
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    const int r = lane + 64 * j;
    if (r < n) G[(int64_t)blockIdx.y * ld * ld + r + (int64_t)c * ld] = make_double2(zr[j], zi[j]);
  }
}

template <int NR>
void launch_back(hipStream_t st, const double* Zt, const double* V, const double* tau, double* G, int n, int count,
                 int c0, int ld) {
  const int cols = n - c0, per = kTrdThreads / 64;
  hipLaunchKernelGGL(k_trd_back<NR>, dim3((unsigned)((cols + per - 1) / per), (unsigned)count), dim3(kTrdThreads), 0,
                     st, Zt, (const double2*)V, (const double2*)tau, (double2*)G, n, c0, ld);
}

// Busy wait of `ticks` ticks of the constant-rate wall clock (one wave).
__global__ void k_spin(long long ticks) {
  const long long t0 = wall_clock64();
  while (wall_clock64() - t0 < ticks) {
  }
}

}  // namespace

int64_t eig_trd_max_n(tdvp_ctx* ctx) {
  // the large variant's LDS: 3 n complex values plus the kernel's own
  // reduction arrays; launches beyond 64 KB are allowed explicitly once
  static int64_t cached[64];
  const int dev = ctx->device;
  if (dev < 0 || dev >= 64) return kTrdMaxN;
  if (cached[dev]) return cached[dev];
  int lim = 0;
  int64_t r = kTrdMaxN;
  const size_t need = sizeof(double2) * 3 * (size_t)kTrdMaxNLarge;
  if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
      (size_t)lim >= need + sizeof(double2) * (kTrdThreads + 8) &&
      hipFuncSetAttribute((const void*)k_trd_multi<(int)(kTrdMaxNLarge / kTrdThreads)>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)need) == hipSuccess)
    r = kTrdMaxNLarge;
  (void)hipGetLastError();
  cached[dev] = r;
  return r;
}

int eig_spin(tdvp_ctx* ctx, hipStream_t st, double microseconds) {
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->device) != hipSuccess || khz <= 0)
    khz = 100000;
  const long long ticks = (long long)(microseconds * 1e-3 * (double)khz);
  hipLaunchKernelGGL(k_spin, dim3(1), dim3(64), 0, st, ticks);
  TDVP_HIP(ctx, hipGetLastError());
  return TDVP_OK;
}

int eig_trd_upload(tdvp_ctx* ctx, hipStream_t st, const TrdSet& set, void* table) {
  if (set.njobs <= 0) return TDVP_OK;
  if (set.njobs > kTrdMaxJobs) return set_error(ctx, TDVP_E_INVALID, "tridiagonal reduction: too many jobs");
  TDVP_HIP(ctx, hipMemcpyAsync(table, set.job, sizeof(TrdJob) * (size_t)set.njobs, hipMemcpyHostToDevice, st));
  return TDVP_OK;
}

int eig_trd_column(tdvp_ctx* ctx, hipStream_t st, const TrdSet& set, const void* table, int64_t k) {
  int64_t blocks = 0, nmax = 0;
  for (int j = 0; j < set.njobs; ++j) {
    const TrdJob& jb = set.job[j];
    if (jb.n <= 0 || jb.n > kTrdMaxNLarge || jb.count <= 0 || jb.lda < jb.n)
      return set_error(ctx, TDVP_E_INVALID, "tridiagonal reduction: size out of range");
    nmax = std::max<int64_t>(nmax, jb.n);
    if (k < jb.n) blocks += (int64_t)jb.count * std::max<int64_t>(1, (jb.n - k - 1 + kTrdRows - 1) / kTrdRows);
  }
  if (set.njobs > kTrdMaxJobs || blocks > INT32_MAX)
    return set_error(ctx, TDVP_E_INVALID, "tridiagonal reduction: too many jobs");
  if (blocks == 0) return TDVP_OK;
  const size_t lds = sizeof(double2) * 3 * (size_t)nmax;
  if (nmax <= kTrdMaxN) {
    hipLaunchKernelGGL(k_trd_multi<(int)(kTrdMaxN / kTrdThreads)>, dim3((unsigned)blocks), dim3(kTrdThreads), lds, st,
                       (const TrdJob*)table, set.njobs, (int)k);
  } else {
    if (nmax > eig_trd_max_n(ctx)) return set_error(ctx, TDVP_E_INVALID, "tridiagonal reduction: size out of range");
    hipLaunchKernelGGL(k_trd_multi<(int)(kTrdMaxNLarge / kTrdThreads)>, dim3((unsigned)blocks), dim3(kTrdThreads),
                       lds, st, (const TrdJob*)table, set.njobs, (int)k);
  }
  TDVP_HIP(ctx, hipGetLastError());
  return TDVP_OK;
}

int eig_trd_back(tdvp_ctx* ctx, hipStream_t st, const double* Zt, const double* V, const double* tau, double* G,
                 int64_t n, int64_t count, int64_t c0, int64_t ld) {
  if (n <= 0 || count <= 0 || c0 >= n) return TDVP_OK;
  if (n > kTrdMaxNLarge || count > 65535 || c0 < 0 || ld < n)
    return set_error(ctx, TDVP_E_INVALID, "tridiagonal back-transformation: size out of range");
  const int ni = (int)n, ci = (int)count, c0i = (int)c0, ldi = (int)ld;
  if (n <= 64) launch_back<1>(st, Zt, V, tau, G, ni, ci, c0i, ldi);
  else if (n <= 128) launch_back<2>(st, Zt, V, tau, G, ni, ci, c0i, ldi);
  else if (n <= 256) launch_back<4>(st, Zt, V, tau, G, ni, ci, c0i, ldi);
  else if (n <= 512) launch_back<8>(st, Zt, V, tau, G, ni, ci, c0i, ldi);
  else if (n <= 768) launch_back<12>(st, Zt, V, tau, G, ni, ci, c0i, ldi);
  else if (n <= 1024) launch_back<16>(st, Zt, V, tau, G, ni, ci, c0i, ldi);
  else launch_back<24>(st, Zt, V, tau, G, ni, ci, c0i, ldi);
  TDVP_HIP(ctx, hipGetLastError());
  return TDVP_OK;
}

}  // namespace tdvp

// FP64 Lanczos vector kernels on complex128 vectors.
//
// The Krylov recurrence, the Gram-Schmidt re-orthogonalisation and the norms
// stay in FP64 whatever precision the block products use.  Reductions are
// two-pass and deterministic: wavefront shuffles, one partial per workgroup
// written to scratch, then one workgroup per result sums the partials in a
// fixed order.  These kernels are HBM-bound (a few bytes per flop), so they
// are written for coalesced 16-byte loads and enough waves to fill 256 CUs.
#include <hip/hip_runtime.h>

#include "ctx.hpp"

namespace tdvp {

namespace {

constexpr int NT = 256;
constexpr int kMaxV = 72;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// block-level sum of (a, b); result valid in thread 0
__device__ __forceinline__ void block_sum2(double& a, double& b) {
  __shared__ double sa[NT / 64], sb[NT / 64];
  a = wave_sum(a);
  b = wave_sum(b);
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    sa[w] = a;
    sb[w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = 0.0;
    b = 0.0;
    for (int i = 0; i < NT / 64; ++i) {
      a += sa[i];
      b += sb[i];
    }
  }
}

// ---- Householder reflection H = I - u u^H (|u|^2 = 2) of batched Hermitian
// n x n matrices (leading dimension ld, consecutive matrices ld^2 apart):
// G -> H G H before an eigensolve, eigenvectors W -> H W after.
// The spectrum is unchanged; a dense u removes exact block structure (zero
// padding, decoupled sectors) that would split the tridiagonal form.
__device__ __forceinline__ double2 reflector_u(int64_t i, int64_t n) {
  const double f = (double)(i + 1) * 0.6180339887498949;   // golden-ratio phases
  const double ph = 6.283185307179586 * (f - floor(f));
  const double r = sqrt(2.0 / (double)n);
  return make_double2(r * cos(ph), r * sin(ph));
}

// p = G u, one workgroup per 64 rows of one matrix (blockIdx.y)
__global__ __launch_bounds__(NT) void k_reflect_p(const double2* __restrict__ G, int64_t n, int64_t ld,
                                                  double2* __restrict__ P) {
  __shared__ double2 part[4][64];
  const double2* A = G + (int64_t)blockIdx.y * ld * ld;
  const int64_t r = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  const int cg = threadIdx.x >> 6;
  double re = 0.0, im = 0.0;
  if (r < n)
    for (int64_t c = cg; c < n; c += 4) {
      const double2 a = A[r + c * ld], u = reflector_u(c, n);
      re += a.x * u.x - a.y * u.y;
      im += a.x * u.y + a.y * u.x;
    }
  part[cg][threadIdx.x & 63] = make_double2(re, im);
  __syncthreads();
  if (cg == 0 && r < n) {
    double2 t = part[0][threadIdx.x];
    for (int q = 1; q < 4; ++q) {
      t.x += part[q][threadIdx.x].x;
      t.y += part[q][threadIdx.x].y;
    }
    P[(int64_t)blockIdx.y * n + r] = t;
  }
}

// w = p - (u^H p / 2) u in place, one workgroup per matrix
__global__ __launch_bounds__(NT) void k_reflect_w(double2* __restrict__ P, int64_t n) {
  double2* p = P + (int64_t)blockIdx.x * n;
  double re = 0.0, im = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += NT) {
    const double2 u = reflector_u(i, n), v = p[i];
    re += u.x * v.x + u.y * v.y;
    im += u.x * v.y - u.y * v.x;
  }
  block_sum2(re, im);
  __shared__ double gamma;
  if (threadIdx.x == 0) gamma = 0.5 * re;   // u^H G u is real for Hermitian G
  __syncthreads();
  const double g = gamma;
  for (int64_t i = threadIdx.x; i < n; i += NT) {
    const double2 u = reflector_u(i, n), v = p[i];
    p[i] = make_double2(v.x - g * u.x, v.y - g * u.y);
  }
}

// G -= u w^H + w u^H over all count matrices
__global__ __launch_bounds__(NT) void k_reflect_update(double2* __restrict__ G, int64_t n, int64_t ld, int64_t count,
                                                       const double2* __restrict__ W) {
  const int64_t nn = n * n, total = nn * count;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int64_t m = e / nn, rc = e - m * nn, c = rc / n, r = rc - c * n;
    const double2 ur = reflector_u(r, n), uc = reflector_u(c, n);
    const double2 wr = W[m * n + r], wc = W[m * n + c];
    double2& g = G[m * ld * ld + r + c * ld];
    double2 a = g;
    // u_r conj(w_c) + w_r conj(u_c)
    a.x -= (ur.x * wc.x + ur.y * wc.y) + (wr.x * uc.x + wr.y * uc.y);
    a.y -= (ur.y * wc.x - ur.x * wc.y) + (wr.y * uc.x - wr.x * uc.y);
    g = a;
  }
}

// columns c >= c0 of each matrix: W_c -= u (u^H W_c); one workgroup per column
__global__ __launch_bounds__(NT) void k_reflect_back(double2* __restrict__ G, int64_t n, int64_t ld, int64_t c0) {
  double2* w = G + (int64_t)blockIdx.y * ld * ld + (c0 + blockIdx.x) * ld;
  double re = 0.0, im = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += NT) {
    const double2 u = reflector_u(i, n), v = w[i];
    re += u.x * v.x + u.y * v.y;
    im += u.x * v.y - u.y * v.x;
  }
  block_sum2(re, im);
  __shared__ double2 d;
  if (threadIdx.x == 0) d = make_double2(re, im);
  __syncthreads();
  const double2 dd = d;
  for (int64_t i = threadIdx.x; i < n; i += NT) {
    const double2 u = reflector_u(i, n), v = w[i];
    w[i] = make_double2(v.x - (u.x * dd.x - u.y * dd.y), v.y - (u.x * dd.y + u.y * dd.x));
  }
}

// Krylov basis vectors are stored as complex128 (double2) or, to halve the
// basis memory, complex64 (float2); they are read and combined in FP64.
__device__ __forceinline__ double2 ldv(const double2* p) { return *p; }
__device__ __forceinline__ double2 ldv(const float2* p) {
  const float2 v = *p;
  return make_double2((double)v.x, (double)v.y);
}
__device__ __forceinline__ void stv(double2* p, double2 v) { *p = v; }
__device__ __forceinline__ void stv(float2* p, double2 v) { *p = make_float2((float)v.x, (float)v.y); }

int nblocks_for(int64_t n) {
  int64_t g = (n + NT * 4 - 1) / (NT * 4);
  if (g < 1) g = 1;
  if (g > 1024) g = 1024;
  return (int)g;
}

// partial[k * G + g] = sum_{i in chunk g} conj(V_k[i]) w[i] for every k < nv,
// or, with d_j (index read on the device), every k <= *d_j.  The vectors go
// in groups of kDotGroup, so each element of w is read once per group (not
// once per vector); every k keeps its own summation order.
constexpr int kDotGroup = 8;
template <typename VT>
__global__ __launch_bounds__(NT) void k_dots_partial(const VT* __restrict__ V, int64_t stride,
                                                     const double2* __restrict__ w, int64_t n,
                                                     double2* __restrict__ partial, const int* __restrict__ d_j,
                                                     int nv) {
  const int g = blockIdx.x, G = gridDim.x;
  const int ke = d_j ? *d_j + 1 : nv;
  int64_t chunk = (n + G - 1) / G;
  int64_t lo = (int64_t)g * chunk, hi = lo + chunk < n ? lo + chunk : n;
  for (int kb = 0; kb < ke; kb += kDotGroup) {
    const int nk = ke - kb < kDotGroup ? ke - kb : kDotGroup;
    double re[kDotGroup], im[kDotGroup];
#pragma unroll
    for (int q = 0; q < kDotGroup; ++q) re[q] = im[q] = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += NT) {
      const double2 b = w[i];
#pragma unroll
      for (int q = 0; q < kDotGroup; ++q) {
        if (q < nk) {
          const double2 a = ldv(V + (int64_t)(kb + q) * stride + i);
          re[q] += a.x * b.x + a.y * b.y;
          im[q] += a.x * b.y - a.y * b.x;
        }
      }
    }
    for (int q = 0; q < nk; ++q) {
      double r = re[q], m = im[q];
      block_sum2(r, m);
      if (threadIdx.x == 0) partial[(int64_t)(kb + q) * G + g] = make_double2(r, m);
      __syncthreads();   // block_sum2's shared slots are reused by the next vector
    }
  }
}

__global__ __launch_bounds__(NT) void k_reduce(const double2* __restrict__ partial, int G,
                                               double* __restrict__ out, const int* __restrict__ d_j) {
  const int k = blockIdx.x;
  if (d_j && k > *d_j) return;
  double re = 0.0, im = 0.0;
  for (int i = threadIdx.x; i < G; i += NT) {
    double2 p = partial[(int64_t)k * G + i];
    re += p.x;
    im += p.y;
  }
  block_sum2(re, im);
  if (threadIdx.x == 0) {
    out[2 * k] = re;
    out[2 * k + 1] = im;
  }
}

// w -= sum_k c_k V_k ; optional partial |w|^2; with d_j, nv = *d_j + 1
template <typename VT>
__global__ __launch_bounds__(NT) void k_sub_combo(double2* __restrict__ w, const VT* __restrict__ V,
                                                  int64_t stride, int nv, const double* __restrict__ coef,
                                                  int64_t n, double2* __restrict__ partial,
                                                  const int* __restrict__ d_j) {
  __shared__ double c[2 * kMaxV];
  if (d_j) nv = *d_j + 1;
  for (int i = threadIdx.x; i < 2 * nv; i += NT) c[i] = coef[i];
  __syncthreads();
  const int g = blockIdx.x, G = gridDim.x;
  int64_t chunk = (n + G - 1) / G;
  int64_t lo = (int64_t)g * chunk, hi = lo + chunk < n ? lo + chunk : n;
  double nrm = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += NT) {
    double2 x = w[i];
    for (int k = 0; k < nv; ++k) {
      double2 v = ldv(V + (int64_t)k * stride + i);
      double cr = c[2 * k], ci = c[2 * k + 1];
      x.x -= cr * v.x - ci * v.y;
      x.y -= cr * v.y + ci * v.x;
    }
    w[i] = x;
    nrm += x.x * x.x + x.y * x.y;
  }
  if (partial) {
    double z = 0.0;
    block_sum2(nrm, z);
    if (threadIdx.x == 0) partial[g] = make_double2(nrm, 0.0);
  }
}

template <typename VT>
__global__ __launch_bounds__(NT) void k_combo(double2* __restrict__ out, const VT* __restrict__ V,
                                              int64_t stride, int nv, const double* __restrict__ coef,
                                              int64_t n) {
  __shared__ double c[2 * kMaxV];
  for (int i = threadIdx.x; i < 2 * nv; i += NT) c[i] = coef[i];
  __syncthreads();
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
    double2 x = make_double2(0.0, 0.0);
    for (int k = 0; k < nv; ++k) {
      double2 v = ldv(V + (int64_t)k * stride + i);
      double cr = c[2 * k], ci = c[2 * k + 1];
      x.x += cr * v.x - ci * v.y;
      x.y += cr * v.y + ci * v.x;
    }
    out[i] = x;
  }
}

__global__ __launch_bounds__(NT) void k_scale_copy(double2* __restrict__ dst, const double2* __restrict__ src,
                                                   double s, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
    double2 x = src[i];
    dst[i] = make_double2(s * x.x, s * x.y);
  }
}

// Next Lanczos vector w / sqrt(b2) into basis slot *d_j + 1 (when it exists)
// and into the fixed operator input x (FP64); b2 = |w|^2 from the device.
template <typename VT>
__global__ __launch_bounds__(NT) void k_advance(VT* __restrict__ V, int64_t stride, double2* __restrict__ x,
                                                const double2* __restrict__ w, int64_t n,
                                                const double* __restrict__ b2, const int* __restrict__ d_j,
                                                int maxdim) {
  const double q = *b2;
  const double s = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
  const int j = *d_j;
  VT* dst = j + 1 < maxdim ? V + (int64_t)(j + 1) * stride : nullptr;
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
    double2 v = w[i];
    v = make_double2(s * v.x, s * v.y);
    x[i] = v;
    if (dst) stv(dst + i, v);
  }
}

// basis slot 0 (complex64) from an FP64 vector
__global__ __launch_bounds__(NT) void k_store32(float2* __restrict__ dst, const double2* __restrict__ src, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) stv(dst + i, src[i]);
}

__global__ void k_set_index(int* __restrict__ d_j, int v, int add) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *d_j = add ? *d_j + v : v;
}

__global__ __launch_bounds__(NT) void k_norm_partial(const double2* __restrict__ x, int64_t n,
                                                     double2* __restrict__ partial) {
  const int g = blockIdx.x, G = gridDim.x;
  int64_t chunk = (n + G - 1) / G;
  int64_t lo = (int64_t)g * chunk, hi = lo + chunk < n ? lo + chunk : n;
  double s = 0.0, nonfinite = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += NT) {
    double2 v = x[i];
    double q = v.x * v.x + v.y * v.y;
    if (!isfinite(v.x) || !isfinite(v.y)) nonfinite += 1.0;
    s += q;
  }
  block_sum2(s, nonfinite);
  if (threadIdx.x == 0) partial[g] = make_double2(s, nonfinite);
}

// out[b] = sum_i conj(x_i) y_i over block b: elements [meta[2b], meta[2b] + meta[2b+1])
__global__ __launch_bounds__(NT) void k_block_dots(const double2* __restrict__ x, const double2* __restrict__ y,
                                                   const int64_t* __restrict__ meta, double2* __restrict__ out) {
  const int64_t off = meta[2 * blockIdx.x], len = meta[2 * blockIdx.x + 1];
  double re = 0.0, im = 0.0;
  for (int64_t i = threadIdx.x; i < len; i += NT) {
    const double2 a = x[off + i], b = y[off + i];
    re += a.x * b.x + a.y * b.y;
    im += a.x * b.y - a.y * b.x;
  }
  block_sum2(re, im);
  if (threadIdx.x == 0) out[blockIdx.x] = make_double2(re, im);
}

// n x n matrix whose leading g x g block is set: the rest becomes the identity
__global__ __launch_bounds__(NT) void k_pad_identity(double2* __restrict__ A, int64_t n, int64_t g) {
  int64_t tot = n * n;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < tot; e += (int64_t)gridDim.x * NT) {
    int64_t i = e % n, j = e / n;
    if (i >= g || j >= g) A[e] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
}

// strictly lower triangle of `count` consecutive n x n matrices set to zero
__global__ __launch_bounds__(NT) void k_zero_lower(double2* __restrict__ A, int64_t n, int64_t count) {
  int64_t tot = n * n * count;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < tot; e += (int64_t)gridDim.x * NT) {
    int64_t r = e % (n * n), i = r % n, j = r / n;
    if (i > j) A[e] = make_double2(0.0, 0.0);
  }
}

// scale[0] = largest |A_ii| of the leading g x g block (one workgroup)
__global__ __launch_bounds__(NT) void k_diag_max(const double2* __restrict__ A, int64_t n, int64_t g,
                                                 double* __restrict__ scale) {
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < g; i += NT) m = fmax(m, fabs(A[i + i * n].x));
  __shared__ double sm[NT];
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) scale[0] = sm[0] > 0.0 ? sm[0] : 1.0;
}

// Padding of an n x n matrix beyond its leading g x g block: distinct values
// v * scale * (1 + (i - g) / n) on the diagonal (no degenerate cluster, and on
// the scale of the block's own eigenvalues), zero elsewhere.
__global__ __launch_bounds__(NT) void k_pad(double2* __restrict__ A, int64_t n, int64_t g, double v,
                                            const double* __restrict__ scale) {
  int64_t tot = n * n;
  const double s = v * scale[0];
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < tot; e += (int64_t)gridDim.x * NT) {
    int64_t i = e % n, j = e / n;
    if (i >= g || j >= g) A[e] = make_double2(i == j ? s * (1.0 + (double)(i - g) / (double)n) : 0.0, 0.0);
  }
}

// A[:, c] *= 1 / sqrt(lam[c]) for c < cols (columns of leading dimension ld)
__global__ __launch_bounds__(NT) void k_scale_cols(double2* __restrict__ A, int64_t ld, int64_t rows, int64_t cols,
                                                   const double* __restrict__ lam) {
  int64_t tot = rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < tot; e += (int64_t)gridDim.x * NT) {
    int64_t r = e % rows, c = e / rows;
    double s = 1.0 / sqrt(lam[c]);
    double2 v = A[r + c * ld];
    A[r + c * ld] = make_double2(s * v.x, s * v.y);
  }
}

int grid_1d(int64_t n) {
  int64_t g = (n + NT - 1) / NT;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

int vec_dots(tdvp_ctx* ctx, const double* V, int64_t stride, int nv, const double* w, int64_t n,
             double* d_out, bool v32) {
  if (nv <= 0) return TDVP_OK;
  int G = nblocks_for(n);
  size_t need = sizeof(double2) * (size_t)G * nv;
  TDVP_HIP(ctx, ctx->ws_vec.ensure(need));
  double2* partial = (double2*)ctx->ws_vec.p;
  if (v32)
    hipLaunchKernelGGL(k_dots_partial<float2>, dim3(G), dim3(NT), 0, ctx->stream, (const float2*)V, stride,
                       (const double2*)w, n, partial, (const int*)nullptr, nv);
  else
    hipLaunchKernelGGL(k_dots_partial<double2>, dim3(G), dim3(NT), 0, ctx->stream, (const double2*)V, stride,
                       (const double2*)w, n, partial, (const int*)nullptr, nv);
  hipLaunchKernelGGL(k_reduce, dim3(nv), dim3(NT), 0, ctx->stream, partial, G, d_out, (const int*)nullptr);
  TDVP_HIP(ctx, hipGetLastError());
  return TDVP_OK;
}

int vec_subtract_combo(tdvp_ctx* ctx, double* w, const double* V, int64_t stride, int nv, const double* d_coef,
                       int64_t n, double* d_norm2, bool v32) {
  if (nv > kMaxV) return TDVP_E_INVALID;
  int G = nblocks_for(n);
  double2* partial = nullptr;
  if (d_norm2) {
    TDVP_HIP(ctx, ctx->ws_vec.ensure(sizeof(double2) * (size_t)G));
    partial = (double2*)ctx->ws_vec.p;
  }
  if (v32)
    hipLaunchKernelGGL(k_sub_combo<float2>, dim3(G), dim3(NT), 0, ctx->stream, (double2*)w, (const float2*)V, stride,
                       nv, d_coef, n, partial, (const int*)nullptr);
  else
    hipLaunchKernelGGL(k_sub_combo<double2>, dim3(G), dim3(NT), 0, ctx->stream, (double2*)w, (const double2*)V,
                       stride, nv, d_coef, n, partial, (const int*)nullptr);
  if (d_norm2)
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(NT), 0, ctx->stream, partial, G, d_norm2, (const int*)nullptr);
  TDVP_HIP(ctx, hipGetLastError());
  return TDVP_OK;
}

int vec_scale_copy(tdvp_ctx* ctx, double* dst, const double* src, double s, int64_t n) {
  hipLaunchKernelGGL(k_scale_copy, dim3(grid_1d(n)), dim3(NT), 0, ctx->stream, (double2*)dst,
                     (const double2*)src, s, n);
  TDVP_HIP(ctx, hipGetLastError());
  return TDVP_OK;
}

int vec_combo(tdvp_ctx* ctx, double* out, const double* V, int64_t stride, int nv, const double* d_coef,
              int64_t n, bool v32) {
  if (nv > kMaxV) return TDVP_E_INVALID;
  if (v32)
    hipLaunchKernelGGL(k_combo<float2>, dim3(grid_1d(n)), dim3(NT), 0, ctx->stream, (double2*)out, (const float2*)V,
                       stride, nv, d_coef, n);
  else
    hipLaunchKernelGGL(k_combo<double2>, dim3(grid_1d(n)), dim3(NT), 0, ctx->stream, (double2*)out,
                       (const double2*)V, stride, nv, d_coef, n);
  TDVP_HIP(ctx, hipGetLastError());
  return TDVP_OK;
}

// ---- one Lanczos iteration with its index j in device memory (d_j), so that
// a single captured graph serves every iteration of an exponential ----------

size_t lanczos_partial_bytes(int64_t n, int maxdim) {
  return sizeof(double2) * (size_t)nblocks_for(n) * (size_t)(maxdim + 1);
}

// two classical Gram-Schmidt passes of W against V_0..V_j: coefficients to
// c1 and c2 (2 * maxdim doubles each), |W|^2 after the second pass to d_norm2
int vec_lanczos_orth_it(tdvp_ctx* ctx, double* W, const double* V, int64_t stride, int maxdim, int64_t n,
                        const int* d_j, double* c1, double* c2, double* d_norm2, void* partial_buf, bool v32) {
  if (maxdim > kMaxV) return TDVP_E_INVALID;
  const int G = nblocks_for(n);
  double2* partial = (double2*)partial_buf;
  double* cs[2] = {c1, c2};
  for (int pass = 0; pass < 2; ++pass) {
    if (v32)
      hipLaunchKernelGGL(k_dots_partial<float2>, dim3(G), dim3(NT), 0, ctx->stream, (const float2*)V, stride,
                         (const double2*)W, n, partial, d_j, 0);
    else
      hipLaunchKernelGGL(k_dots_partial<double2>, dim3(G), dim3(NT), 0, ctx->stream, (const double2*)V, stride,
                         (const double2*)W, n, partial, d_j, 0);
    hipLaunchKernelGGL(k_reduce, dim3(maxdim), dim3(NT), 0, ctx->stream, partial, G, cs[pass], d_j);
    if (v32)
      hipLaunchKernelGGL(k_sub_combo<float2>, dim3(G), dim3(NT), 0, ctx->stream, (double2*)W, (const float2*)V,
                         stride, 0, (const double*)cs[pass], n, pass == 1 ? partial : nullptr, d_j);
    else
      hipLaunchKernelGGL(k_sub_combo<double2>, dim3(G), dim3(NT), 0, ctx->stream, (double2*)W, (const double2*)V,
                         stride, 0, (const double*)cs[pass], n, pass == 1 ? partial : nullptr, d_j);
  }
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(NT), 0, ctx->stream, partial, G, d_norm2, (const int*)nullptr);
  TDVP_HIP(ctx, hipGetLastError());
  return TDVP_OK;
}

// x = V_{j+1} = W / sqrt(b2) (the basis slot only while j + 1 < maxdim), then j += 1
int vec_lanczos_advance_it(tdvp_ctx* ctx, double* V, int64_t stride, double* x, const double* W, int64_t n,
                           const double* d_b2, int* d_j, int maxdim, bool v32) {
  if (v32)
    hipLaunchKernelGGL(k_advance<float2>, dim3(grid_1d(n)), dim3(NT), 0, ctx->stream, (float2*)V, stride,
                       (double2*)x, (const double2*)W, n, d_b2, (const int*)d_j, maxdim);
  else
    hipLaunchKernelGGL(k_advance<double2>, dim3(grid_1d(n)), dim3(NT), 0, ctx->stream, (double2*)V, stride,
                       (double2*)x, (const double2*)W, n, d_b2, (const int*)d_j, maxdim);
  hipLaunchKernelGGL(k_set_index, dim3(1), dim3(64), 0, ctx->stream, d_j, 1, 1);
  TDVP_HIP(ctx, hipGetLastError());
  return TDVP_OK;
}

int vec_store_basis32(tdvp_ctx* ctx, double* V32, const double* x, int64_t n) {
  hipLaunchKernelGGL(k_store32, dim3(grid_1d(n)), dim3(NT), 0, ctx->stream, (float2*)V32, (const double2*)x, n);
  TDVP_HIP(ctx, hipGetLastError());
  return TDVP_OK;
}

int vec_set_index(tdvp_ctx* ctx, int* d_j, int v) {
  hipLaunchKernelGGL(k_set_index, dim3(1), dim3(64), 0, ctx->stream, d_j, v, 0);
  TDVP_HIP(ctx, hipGetLastError());
  return TDVP_OK;
}

// d_out[0] = |x|^2, d_out[1] = number of non-finite entries
int vec_norm2(tdvp_ctx* ctx, const double* x, int64_t n, double* d_out) {
  int G = nblocks_for(n);
  TDVP_HIP(ctx, ctx->ws_vec.ensure(sizeof(double2) * (size_t)G));
  double2* partial = (double2*)ctx->ws_vec.p;
  hipLaunchKernelGGL(k_norm_partial, dim3(G), dim3(NT), 0, ctx->stream, (const double2*)x, n, partial);
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(NT), 0, ctx->stream, partial, G, d_out, (const int*)nullptr);
  TDVP_HIP(ctx, hipGetLastError());
  return TDVP_OK;
}

int vec_block_dots(tdvp_ctx* ctx, const double* x, const double* y, const int64_t* d_meta, int nblocks,
                   double* d_out) {
  if (nblocks <= 0) return TDVP_OK;
  hipLaunchKernelGGL(k_block_dots, dim3(nblocks), dim3(NT), 0, ctx->stream, (const double2*)x, (const double2*)y,
                     d_meta, (double2*)d_out);
  TDVP_HIP(ctx, hipGetLastError());
  return TDVP_OK;
}

int vec_pad_identity(tdvp_ctx* ctx, double* A, int64_t n, int64_t g) {
  if (g >= n) return TDVP_OK;
  hipLaunchKernelGGL(k_pad_identity, dim3(grid_1d(n * n)), dim3(NT), 0, ctx->stream, (double2*)A, n, g);
  TDVP_HIP(ctx, hipGetLastError());
  return TDVP_OK;
}

int vec_zero_lower(tdvp_ctx* ctx, double* A, int64_t n, int64_t count) {
  if (n <= 1 || count <= 0) return TDVP_OK;
  hipLaunchKernelGGL(k_zero_lower, dim3(grid_1d(n * n * count)), dim3(NT), 0, ctx->stream, (double2*)A, n, count);
  TDVP_HIP(ctx, hipGetLastError());
  return TDVP_OK;
}

int vec_scale_cols_rsqrt(tdvp_ctx* ctx, double* A, int64_t ld, int64_t rows, int64_t cols, const double* lam) {
  if (rows <= 0 || cols <= 0) return TDVP_OK;
  hipLaunchKernelGGL(k_scale_cols, dim3(grid_1d(rows * cols)), dim3(NT), 0, ctx->stream, (double2*)A, ld, rows, cols,
                     lam);
  TDVP_HIP(ctx, hipGetLastError());
  return TDVP_OK;
}

int vec_reflect_forward(tdvp_ctx* ctx, hipStream_t st, double* G, int64_t n, int64_t count, double* P, int64_t ld) {
  if (n <= 1 || count <= 0) return TDVP_OK;
  if (ld <= 0) ld = n;
  hipLaunchKernelGGL(k_reflect_p, dim3((unsigned)((n + 63) / 64), (unsigned)count), dim3(NT), 0, st,
                     (const double2*)G, n, ld, (double2*)P);
  hipLaunchKernelGGL(k_reflect_w, dim3((unsigned)count), dim3(NT), 0, st, (double2*)P, n);
  hipLaunchKernelGGL(k_reflect_update, dim3(grid_1d(n * n * count)), dim3(NT), 0, st, (double2*)G, n, ld, count,
                     (const double2*)P);
  TDVP_HIP(ctx, hipGetLastError());
  return TDVP_OK;
}

int vec_reflect_back(tdvp_ctx* ctx, hipStream_t st, double* G, int64_t n, int64_t count, int64_t c0, int64_t ld) {
  if (n <= 1 || count <= 0 || c0 >= n) return TDVP_OK;
  if (ld <= 0) ld = n;
  hipLaunchKernelGGL(k_reflect_back, dim3((unsigned)(n - c0), (unsigned)count), dim3(NT), 0, st, (double2*)G, n, ld,
                     c0);
  TDVP_HIP(ctx, hipGetLastError());
  return TDVP_OK;
}

int vec_pad_matrix(tdvp_ctx* ctx, double* A, int64_t n, int64_t g, double v, double* d_scale) {
  if (g >= n) return TDVP_OK;
  hipLaunchKernelGGL(k_diag_max, dim3(1), dim3(NT), 0, ctx->stream, (const double2*)A, n, g, d_scale);
  hipLaunchKernelGGL(k_pad, dim3(grid_1d(n * n)), dim3(NT), 0, ctx->stream, (double2*)A, n, g, v,
                     (const double*)d_scale);
  TDVP_HIP(ctx, hipGetLastError());
  return TDVP_OK;
}

}  // namespace tdvp

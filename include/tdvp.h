/*
 * tdvp.h -- C ABI of the MI355X (gfx950) two-site TDVP hot path for the
 * U(1)_spin x SU(2)_charge symmetric 1D Fermi-Hubbard chain.
 *
 * Paper: two-site TDVP of a U(1)xSU(2)-reduced MPS; each sweep step merges
 * two sites, exponentiates the local effective Hamiltonian with an adaptive
 * Krylov method, splits by SVD and updates the environments (supplementary
 * sections S2.1-S2.3).  This library computes those steps on one GPU.
 *
 * ---------------------------------------------------------------------------
 * Conventions (shared with the CPU oracle by this text only)
 * ---------------------------------------------------------------------------
 * Hamiltonian.  Eq. (1) on an open chain of L sites, with the interaction in
 * its particle-hole symmetric form U (n_up - 1/2)(n_dn - 1/2): that form
 * commutes with the eta-pairing pseudospin of section S2.1, Eq. (1)'s own
 * U n_up n_dn does not ([H, T+] = U T+).  At half filling the two differ by
 * the constant U L / 4, i.e. a global phase.  Sites are numbered 1..L.
 *
 * Labels.  A bond sector is (q, tj): q = 2 S^z and tj = 2T (pseudospin) of
 * everything left of the bond; its degeneracy is dim.  The local multiplets
 * of site k are s = 0: (q=0, tj=1) with components m=+1/2 -> |up dn>,
 * m=-1/2 -> (-1)^k |0>; s = 1: (q=+1, tj=0) = |up>; s = 2: (q=-1, tj=0) = |dn>
 * (Jordan-Wigner mode order 1up, 1dn, 2up, ...; |up dn> = c+_up c+_dn |0>).
 *
 * Reduced tensors (Wigner-Eckart, section S2.1 bond decomposition), with
 * Condon-Shortley coefficients C(j1 m1; j2 m2 | J M):
 *   one-site key (ia, s, ib), block d_a x d_b:
 *     A  (left-canonical):  A_full = A C(ja ma; js mu | jb mb)
 *     B  (right-canonical): B_full = B C(..) sqrt((2ja+1)/(2jb+1))
 *     C1 (one-site centre): C_full = C C(..) / sqrt(2jb+1)
 *   two-site key (ia, s1, tjx, s2, ib), block d_a x d_b, tree ((a s1)->x) s2->b:
 *     Th_full = Th sum_mx C(ja ma; js1 mu1 | jx mx) C(jx mx; js2 mu2 | jb mb) / sqrt(2jb+1)
 *   With A left and B right of the centre, the flat Frobenius inner product of
 *   centre tensors equals the inner product of the states.
 *   environment key (iout, w, iin), block d_out x d_in, channel w = 0 'H'
 *   (scalar), 1 'D+' (tj=1, q=+1), 2 'D-' (tj=1, q=-1):
 *     E_full[(out m'), kappa, (in m)] = E C(j_in m; j_w kappa | j_out m')
 *   Left environment at bond k: <Phi'| O |Phi> over the block of sites 1..k,
 *   O = block Hamiltonian ('H'), or the edge doublets of site k times the site
 *   parity: D+ = (c+_up P, (-1)^k c_dn P), D- = (c+_dn P, -(-1)^k c_up P).
 *   Right environment at bond k: <Psi'| Q |Psi> over sites k+1..L, Q = block
 *   Hamiltonian, or on site k+1: Q^{D+}_kappa = eps(kappa) [D-]_{-kappa},
 *   Q^{D-}_kappa = eps(kappa) [D+]_{-kappa}, eps(+1/2) = 1, eps(-1/2) = -1.
 *   The identity channels are implicit (canonical gauge).
 *
 * Memory.  Block data is complex128, interleaved (re, im), each block
 * column-major with leading dimension = its row count, at the element
 * offset given for it.  Data pointers passed to compute calls are DEVICE
 * pointers owned by the caller; descriptor arrays are HOST pointers read
 * during the call only.  Block order is free, but keys must be unique and
 * offsets must not overlap; the *_layout queries give a canonical layout.
 *
 * Device memory.  Every device buffer the library itself needs (workspaces,
 * the Krylov basis, program arrays, the blocks of a library-owned MPS) comes
 * from the allocator given to tdvp_ctx_create (dev_alloc / dev_free with the
 * caller's `user` pointer), or from hipMalloc / hipFree when none is given
 * (tdvp_env_update_noalloc excepted: it uses a static device array).
 * The library may release a buffer while work that used it is still queued
 * on the context stream: the allocator must order reuse on that stream (a
 * stream-ordered caching allocator bound to the context stream, such as
 * torch's, does).  The callbacks must stay valid until the context and every
 * MPS made with it are destroyed.  dev_alloc returning NULL makes the call
 * that needed the memory fail with TDVP_E_NOMEM.  The batched eigensolver
 * library behind tdvp_sweep / tdvp_split keeps its own small workspace.
 *
 * Errors.  Every call returns TDVP_OK or a negative code and never throws;
 * tdvp_last_error() gives a message.  Work is enqueued on the context stream;
 * heff_apply and env_update do not synchronise.  krylov_expm, split and the
 * sweeps synchronise (they need scalars on the host) and report earlier
 * asynchronous device faults as TDVP_E_HIP.  Every block product marks a
 * device flag when it writes a non-finite value; the next synchronising call
 * (tdvp_ctx_synchronize included) returns TDVP_E_NONFINITE and clears it.
 * A context is not thread-safe; one context per stream.
 */
#ifndef TDVP_H
#define TDVP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  TDVP_OK = 0,
  TDVP_E_INVALID = -1,   /* bad argument (null pointer, bad site, bad enum) */
  TDVP_E_SHAPE = -2,     /* block dims / offsets inconsistent with the bonds */
  TDVP_E_SECTOR = -3,    /* a block key violates the fusion rules or repeats */
  TDVP_E_NOMEM = -4,     /* device or workspace allocation failed */
  TDVP_E_HIP = -5,       /* HIP runtime error (including earlier async faults) */
  TDVP_E_NOCONV = -6,    /* Krylov did not reach the tolerance within maxdim */
  TDVP_E_NONFINITE = -7  /* NaN or Inf met in the data */
};

/* Arithmetic of the block contractions (effective-Hamiltonian applies and
 * environment updates).  TDVP_FP32: FP32 operands and accumulation.
 * TDVP_BF16X3: each operand value split into three bfloat16 slices (once per
 * operand buffer and launch, into a workspace of 16 bytes per complex
 * element), the six leading slice products of every real product
 * accumulated in FP32 (about FP32 accuracy on the bfloat16 matrix cores).  In both reduced modes the
 * block-Hamiltonian environment channels are shifted by their mean diagonal
 * and the shift is added back exactly.  Lanczos scalars, reorthogonalisation,
 * the small exponential, the SVD/QR splits and all local terms stay in FP64 in
 * every mode. */
enum { TDVP_FP64 = 0, TDVP_FP32 = 1, TDVP_BF16X3 = 2 };

typedef struct tdvp_ctx tdvp_ctx;
typedef struct tdvp_mps tdvp_mps;

/* Fermi-Hubbard chain: hopping t (Eq. (1)'s t_h), interaction U, L sites. */
typedef struct {
  double t;
  double U;
  int32_t L;
} tdvp_model;

/* One bond: n sectors (q[i], tj[i]) of degeneracy dim[i] (host arrays). */
typedef struct {
  int32_t n;
  const int32_t* q;
  const int32_t* tj;
  const int64_t* dim;
} tdvp_bond;

/* Block-sparse reduced tensor: nblocks keys (3 or 5 ints each, host),
 * element offsets (host), device data of `size` complex128 elements. */
typedef struct {
  int32_t nblocks;
  const int32_t* keys;
  const int64_t* offsets;
  void* data;
  int64_t size;
} tdvp_blocks;

typedef struct {
  int32_t iters;        /* Krylov dimension used */
  int32_t converged;    /* 1 if the error estimate met tol (or breakdown) */
  double err_est;       /* beta_m |[exp(tau T_m)]_{m,1}| |x| */
  double norm_in;       /* |x| on entry */
  double alpha[64];     /* Lanczos diagonal (first min(iters,64)) */
  double beta[64];      /* Lanczos off-diagonal */
  int32_t graph_iters;  /* iterations replayed from the captured iteration graph */
} tdvp_krylov_info;

typedef struct {
  double eps_tol;        /* discarded weight tolerance (relative), e.g. 1e-4 */
  int64_t chi_cap;       /* cap on sum_kept (2j+1) d per bond (full-state units) */
  int32_t keep_all;      /* 1: keep every singular value, zero ones included */
  double krylov_tol;     /* Lanczos tolerance, relative to |x| */
  int32_t krylov_maxdim; /* maximal Krylov dimension (<= 64) */
} tdvp_trunc;

typedef struct {
  double max_discarded;   /* largest discarded weight of one bond update */
  double sum_discarded;   /* sum over the sweep */
  int64_t max_chi;        /* largest full-state bond dimension after the sweep */
  int64_t max_chi_su2;    /* largest sum of degeneracies */
  int32_t krylov_iters;   /* total Lanczos iterations (two- and one-site) */
  int32_t krylov_max;     /* largest Krylov dimension used */
  int32_t nonconverged;   /* exponentials that hit maxdim */
  double heff_flops;      /* algorithmic flops of all H_eff applies */
  double env_flops;       /* algorithmic flops of all environment updates */
  double seconds;         /* host wall time of the call */
  double t_heff, t_lanczos, t_svd, t_env;  /* seconds per phase (device events) */
  int32_t graph_iters;    /* Lanczos iterations replayed from captured graphs */
  int32_t eig_fallbacks;  /* sector Gram matrices re-solved by the Jacobi-based fallback */
} tdvp_sweep_info;

/* Plan of one H_eff apply, exported for host-side inspection and tests.
 * kind 0: y[out] += coef * E[env] . x[in]   (left-environment term)
 * kind 1: y[out] += coef * x[in] . E[env]^T (right-environment term)
 * kind 2: y[out] += coef * x[in]            (local term)               */
typedef struct {
  int32_t kind;
  int32_t out;
  int32_t in;
  int32_t env;
  double coef;
} tdvp_term;

/* Plan of one environment update (host inspection):
 * kind 0: out[o] += coef * op(bra[b])^ . E[env] . op(ket[k])
 * kind 1: out[o] += coef * op(bra[b])^ . op(ket[k])    (identity channel)
 * For direction +1 op(bra)^ = A^dag, op(ket) = A; for -1 op(bra)^ = conj(B),
 * op(ket) = B^T. */
typedef struct {
  int32_t kind;
  int32_t out;
  int32_t bra;
  int32_t ket;
  int32_t env;
  double coef;
} tdvp_env_term;

/* ---- context -------------------------------------------------------------
 * device: HIP device ordinal; hip_stream: hipStream_t or NULL (the library
 * then creates its own default-priority, non-blocking stream, which is not
 * ordered with any other stream, the null stream included: a caller whose
 * inputs come from kernels on another stream passes that stream here or
 * synchronises first); precision: TDVP_FP64/FP32/BF16X3 (the precision
 * ladder of the block products, supplementary section S2.5 for float32);
 * dev_alloc / dev_free / user: the device allocator (both NULL: hipMalloc).
 * Errors: INVALID (bad ordinal, precision, or only one callback), HIP (no
 * device), NOMEM. */
int tdvp_ctx_create(tdvp_ctx** out, int32_t device, void* hip_stream, int32_t precision,
                    void* (*dev_alloc)(size_t bytes, void* user), void (*dev_free)(void* ptr, void* user),
                    void* user);
void tdvp_ctx_destroy(tdvp_ctx* ctx);
int tdvp_ctx_set_precision(tdvp_ctx* ctx, int32_t precision);
/* Splitting of long K chains in effective-Hamiltonian launches: every output
 * tile whose chain is longer than alpha x the mean work per resident
 * workgroup is cut into pieces of at least kmin steps of depth, summed by a
 * second kernel in a fixed order (results stay deterministic; the pieces sum
 * in another order than the unsplit chain, so FP64 results differ in the last
 * bits).  alpha < 0: the size rule (split only applies of >= 1e11 flops, alpha
 * 1, kmin 128; environment updates never); alpha >= 0 (0: never) applies to
 * applies and environment updates alike.  Applies to programs built
 * afterwards.  Errors: INVALID. */
int tdvp_ctx_set_split(tdvp_ctx* ctx, double alpha, int32_t kmin);
/* Storage of the Krylov basis (the memory side of supplementary section
 * S2.3, where float32 halves the memory of the largest runs): TDVP_FP64
 * (default) or TDVP_FP32 (complex64 basis vectors, half the memory).  With
 * FP32 storage the recurrence keeps an FP64 copy of the current vector (the
 * operator input), and the Lanczos scalars, the operator applies and the
 * working vector stay FP64; the re-orthogonalisation and the final
 * combination read the rounded basis (relative error of the result about
 * 1e-7).  Applies to later Krylov exponentials (tdvp_krylov_expm and the
 * sweeps).  Errors: INVALID. */
int tdvp_ctx_set_krylov_storage(tdvp_ctx* ctx, int32_t precision);
/* Host staging in sweeps (supplementary section S2.3 stores the state on the
 * CPU and keeps only the tensors being worked on in GPU memory): with enable
 * = 1, tdvp_sweep moves every MPS tensor and environment that the next bond
 * update does not read to pinned host memory after each bond (copies on the
 * context stream; the device memory goes back to the allocator) and brings
 * those of the next bond back before it.  Results are bit-identical to an
 * unstaged sweep.  Calls that read the whole chain (measure, overlap,
 * site_read, tdvp_sweep1) bring everything back first.  Errors: INVALID. */
int tdvp_ctx_set_host_staging(tdvp_ctx* ctx, int32_t enable);
/* Device memory held through the context's allocator (by the context and the
 * MPS made with it): *live_bytes now, *peak_bytes the high-water mark since
 * the last reset; reset_peak = 1 then sets the mark to the live value.
 * Host-only query (no device call).  Errors: INVALID. */
int tdvp_ctx_memory(tdvp_ctx* ctx, int64_t* live_bytes, int64_t* peak_bytes, int32_t reset_peak);
/* Graph replay of Lanczos iterations (enable 1, the default unless the
 * environment variable TDVP_GRAPH is 0, or 0).  With it on, each Krylov
 * exponential of an effective Hamiltonian records one iteration (apply, two
 * Gram-Schmidt passes, norm, copy of the coefficients to the host, next basis
 * vector) as a HIP graph, once the tiling autotuner has settled, and replays
 * it for every further iteration; the iteration index lives in device memory.
 * Results are identical either way.  Errors: INVALID (null ctx). */
int tdvp_ctx_set_graphs(tdvp_ctx* ctx, int32_t enable);
/* Waits for the context stream; HIP (earlier asynchronous fault) or
 * NONFINITE (an earlier launch wrote non-finite values). */
int tdvp_ctx_synchronize(tdvp_ctx* ctx);
/* Last error message of ctx, or of the calling thread when ctx is NULL. */
const char* tdvp_last_error(const tdvp_ctx* ctx);

/* ---- layouts (host only, no GPU needed) ----------------------------------
 * Canonical block list of a centre tensor between bonds left and right:
 * nsites = 2 -> keys (ia, s1, tjx, s2, ib); nsites = 1 -> keys (ia, s, ib).
 * Two-call pattern: pass keys = offsets = NULL to get *nblocks and *total. */
int tdvp_center_layout(const tdvp_bond* left, const tdvp_bond* right, int32_t nsites,
                       int32_t* nblocks, int32_t* keys, int64_t* offsets, int64_t* total);
/* Canonical block list of an environment on `bond`: all (iout, w, iin)
 * allowed by the selection rules of channel w. */
int tdvp_env_layout(const tdvp_bond* bond, int32_t* nblocks, int32_t* keys, int64_t* offsets,
                    int64_t* total);

/* ---- effective Hamiltonian -----------------------------------------------
 * The map whose exponential TDVP takes at every step (supplementary section
 * S2.2; the environment and Krylov contractions that dominate the cost are
 * those of section S2.3): the Hamiltonian of Eq. (1) projected on the block
 * of sites site..site+nsites-1 (nsites 1 or 2) between the left and right
 * environments.  y = H_eff x for that block:
 * left = bond site-1, right = bond site+nsites-1, Lenv = left environment at
 * bond site-1, Renv = right environment at bond site+nsites-1.  x and y must
 * list the same keys (offsets may differ); y is overwritten.
 * The left-environment block products, the local two-site terms with their
 * recoupling coefficients and the right-environment block products are fused
 * in one grouped-GEMM launch.  x and y are caller-owned device buffers; y
 * must not overlap x or the environments.  Does not synchronise.  Errors:
 * INVALID (null pointer, bad site), SHAPE / SECTOR (descriptors inconsistent
 * with the bonds), NOMEM; non-finite output surfaces at the next
 * synchronising call as NONFINITE. */
int tdvp_heff_apply(tdvp_ctx* ctx, const tdvp_model* model, int32_t site, int32_t nsites,
                    const tdvp_bond* left, const tdvp_bond* right, const tdvp_blocks* Lenv,
                    const tdvp_blocks* Renv, const tdvp_blocks* x, tdvp_blocks* y);

/* Host-side plan of the same apply (no GPU; the sector bookkeeping and
 * Wigner-Eckart recoupling of supplementary section S2.1): fills up to *nterms terms and
 * sets *nterms to the count (terms may be NULL) and *flops to the algorithmic
 * flop count (8 per complex multiply-add of every block product). */
int tdvp_heff_plan(const tdvp_model* model, int32_t site, int32_t nsites, const tdvp_bond* left,
                   const tdvp_bond* right, const tdvp_blocks* Lenv, const tdvp_blocks* Renv,
                   const tdvp_blocks* x, int64_t* nterms, tdvp_term* terms, double* flops);

/* ---- Krylov exponential --------------------------------------------------
 * The local evolution of supplementary section S2.2 (a Krylov matrix
 * exponential whose dimension is chosen adaptively):
 * x <- exp(tau H_eff) x, tau = tau_re + i tau_im (TDVP uses tau = -i dt/2
 * forward and +i dt/2 for the one-site backward step).  Lanczos with full
 * FP64 classical Gram-Schmidt re-orthogonalisation (two passes); stops when
 * beta_m |[exp(tau T_m)]_{m,1}| <= tol |x|, on breakdown, or at maxdim
 * (then TDVP_E_NOCONV with the best iterate, the maxdim-dimensional Krylov
 * approximation, left in x).  x is a caller-owned device buffer, updated in
 * place; info (optional, host) receives the recurrence.  Synchronises.
 * Errors: INVALID (maxdim outside 1..64, tol < 0), NOCONV, NONFINITE (x or
 * the applies not finite), NOMEM, HIP. */
int tdvp_krylov_expm(tdvp_ctx* ctx, const tdvp_model* model, int32_t site, int32_t nsites,
                     const tdvp_bond* left, const tdvp_bond* right, const tdvp_blocks* Lenv,
                     const tdvp_blocks* Renv, tdvp_blocks* x, double tau_re, double tau_im,
                     double tol, int32_t maxdim, tdvp_krylov_info* info);

/* Host helper used by krylov_expm, exported for tests (the small exponential
 * of the adaptive Krylov step, supplementary section S2.2): y = nrm exp(tau T)
 * e_1 for the real symmetric tridiagonal T with diagonal alpha[0..n) and
 * off-diagonal beta[0..n-1); y is n complex numbers, interleaved.  Host
 * arrays.  Errors: INVALID, NOCONV (tridiagonal eigensolver). */
int tdvp_tridiag_expm(int32_t n, const double* alpha, const double* beta, double tau_re, double tau_im,
                      double nrm, double* y);

/* ---- environment update ----------------------------------------------------
 * The environment recursion that accompanies every sweep step (supplementary
 * sections S2.2-S2.3; L_i = A^dag (L_{i-1} x W_i) A and its mirror image).
 * direction +1: env_in = left environment at bond site-1 (bond_in), tensor =
 *   left-canonical A of `site` with keys (ia on bond_in, s, ib on bond_out);
 *   env_out = left environment at bond site (bond_out).
 * direction -1: env_in = right environment at bond site (bond_in), tensor =
 *   right-canonical B of `site` with keys (ia on bond_out, s, ib on bond_in);
 *   env_out = right environment at bond site-1 (bond_out).
 * env_out keys must be those of tdvp_env_layout(bond_out); it is overwritten.
 * All data are caller-owned device buffers; env_out must not overlap the
 * inputs.  Does not synchronise.  Errors as tdvp_heff_apply. */
int tdvp_env_update(tdvp_ctx* ctx, const tdvp_model* model, int32_t site, int32_t direction,
                    const tdvp_bond* bond_in, const tdvp_bond* bond_out, const tdvp_blocks* env_in,
                    const tdvp_blocks* tensor, tdvp_blocks* env_out);
/* Allocation-free variant, for callers that cannot allocate device memory
 * (code under stream capture, serving loops that forbid hipMalloc): the same
 * arguments, layouts, results (bit-identical for the same precision and
 * inputs) and errors as tdvp_env_update, but every device buffer beyond the
 * caller's inputs and outputs -- the stage-1 products E . op(ket), the
 * program arrays, the shifts of reduced-precision launches, the partial sums
 * of split K chains -- lives in one static device array of 64 MiB per device,
 * held from the first context created on that device until the process ends.
 * The call allocates no device or pinned host memory (the program arrays are
 * copied from host memory kept by the context, on the context stream).
 * Limits: stage-1 products plus partial sums up to 60 MiB (33 MB at a
 * chi = 4096 bond with Table-S2-shaped sectors), program arrays up to about
 * 4 MiB; beyond them TDVP_E_NOMEM with nothing launched.  Every call on a
 * device shares its array and overwrites it: calls that overlap on one device
 * (other contexts, streams or threads) race.  Split-BF16 precision is not
 * available here (TDVP_E_INVALID): its operand slices need a workspace of
 * the size of the operands.  Does not synchronise. */
int tdvp_env_update_noalloc(tdvp_ctx* ctx, const tdvp_model* model, int32_t site, int32_t direction,
                            const tdvp_bond* bond_in, const tdvp_bond* bond_out, const tdvp_blocks* env_in,
                            const tdvp_blocks* tensor, tdvp_blocks* env_out);
/* Host-side plan of the same update (no GPU): terms as tdvp_env_term, flop
 * count as tdvp_heff_plan.  Two-call pattern on *nterms. */
int tdvp_env_plan(const tdvp_model* model, int32_t site, int32_t direction, const tdvp_bond* bond_in,
                  const tdvp_bond* bond_out, const tdvp_blocks* env_in, const tdvp_blocks* tensor,
                  const tdvp_blocks* env_out, int64_t* nterms, tdvp_env_term* terms, double* flops);

/* ---- MPS and sweep ----------------------------------------------------------
 * The state that TDVP evolves: an MPS in the reduced U(1) x SU(2) form of
 * supplementary section S2.1.  tdvp_mps_create copies a right-canonical MPS
 * (centre C1 on site 1, B on sites 2..L; bonds[0..L], sites[0..L-1] with keys
 * (ia, s, ib) on bonds[k-1], bonds[k]; device data, read only during the
 * call) into library-owned memory (the context's allocator) and builds the
 * right environments.  tdvp_mps_create_neel builds the Neel state of Eq. (2)
 * (up on odd sites); complete = 1 pads every bond to its full symmetric
 * dimension (zero-weight directions), which makes two-site TDVP exact.
 * Errors: INVALID, SHAPE, SECTOR (boundary bonds must be the vacuum (0, 0)
 * of dimension 1), NOMEM, HIP. */
int tdvp_mps_create(tdvp_ctx* ctx, const tdvp_model* model, const tdvp_bond* bonds,
                    const tdvp_blocks* sites, tdvp_mps** out);
int tdvp_mps_create_neel(tdvp_ctx* ctx, const tdvp_model* model, int32_t complete, tdvp_mps** out);
/* Releases the MPS; safe after its context has been destroyed. */
void tdvp_mps_destroy(tdvp_mps* mps);
/* bond k in 0..L: sector count, and (if arrays non-NULL) the sectors. */
int tdvp_mps_bond(const tdvp_mps* mps, int32_t k, int32_t* n, int32_t* q, int32_t* tj, int64_t* dim);
/* site tensor k in 1..L: layout query (two-call pattern) and host copy. */
int tdvp_mps_site_layout(const tdvp_mps* mps, int32_t k, int32_t* nblocks, int32_t* keys,
                         int64_t* offsets, int64_t* total);
int tdvp_mps_site_read(tdvp_ctx* ctx, const tdvp_mps* mps, int32_t k, void* host_dst);
/* One time step dt of symmetric second-order two-site TDVP (supplementary
 * section S2.2; truncation by discarded weight, section S2.4): left-to-right
 * then right-to-left with tau = dt/2 each, every bond merged, evolved by
 * exp(-i tau H2), split by per-sector SVD (truncation: whole multiplets by
 * descending singular value while the discarded weight stays within
 * eps_tol of the total and the kept full dimension within chi_cap; kept
 * values renormalised), environments updated and the one-site centre evolved
 * back by exp(+i tau H1).  The MPS returns to right-canonical form.  The
 * library reallocates the MPS and environment blocks as bonds change, through
 * the context's allocator.  Synchronises.  Errors: INVALID (null, foreign or
 * split-result MPS, bad trunc), NONFINITE, NOMEM, HIP, NOCONV (eigensolver);
 * Krylov exponentials that reach maxdim are counted in info, not errors. */
int tdvp_sweep(tdvp_ctx* ctx, tdvp_mps* mps, double dt, const tdvp_trunc* trunc,
               tdvp_sweep_info* info);

/* ---- two-site split ---------------------------------------------------------
 * The SVD step of a two-site update as a call of its own (supplementary
 * section S2.2; truncated weight, section S2.4): per coupled sector x of the
 * bond between the two sites, the matrix M_x with rows (a, s1) and columns
 * (s2, b) of theta is decomposed, whole multiplets are kept by the rule of
 * tdvp_sweep (eps_tol, chi_cap; keep_all keeps every value, zeros included),
 * and theta = A . C (direction +1: A left-canonical on site 1, the centre on
 * site 2) or C . B (direction -1: centre on site 1, B right-canonical on
 * site 2), with the kept values renormalised to the norm of theta.
 * tdvp_split_sectors (host only, two-call pattern): the coupled sectors in
 * the order the singular values are reported, ascending (q, 2j), with the
 * sizes of M_x.  tdvp_split: left/right bonds and theta (device, keys of
 * tdvp_center_layout with nsites 2; not modified).  *out receives a
 * two-site MPS object holding the result (bond 1 = the new bond, site 1 and
 * site 2 the two tensors; read with tdvp_mps_bond / tdvp_mps_site_layout /
 * tdvp_mps_site_read, release with tdvp_mps_destroy; sweeps, measurements
 * and overlaps reject it).  svals (host, optional): sum over sectors of
 * min(rows, cols) doubles, each sector's reduced singular values in
 * descending order, before truncation (computed from the Gram matrix of the
 * smaller side: absolute accuracy about 1e-16 of the largest squared
 * value).  discarded (optional): discarded weight / total weight.
 * Synchronises.  Errors: INVALID, SHAPE, SECTOR, NONFINITE (theta not
 * finite), NOMEM, HIP, NOCONV (eigensolver). */
int tdvp_split_sectors(const tdvp_bond* left, const tdvp_bond* right, int32_t* nsec, int32_t* q, int32_t* tj,
                       int64_t* rows, int64_t* cols);
int tdvp_split(tdvp_ctx* ctx, const tdvp_bond* left, const tdvp_bond* right, const tdvp_blocks* theta,
               int32_t direction, const tdvp_trunc* trunc, tdvp_mps** out, double* svals, double* discarded);

/* One time step dt of symmetric second-order one-site TDVP (supplementary
 * section S2.2: once the bond dimensions have saturated the single-site
 * projector splitting needs no SVD): left to right with tau = dt/2 every
 * centre is evolved by exp(-i tau H1), moved on by a QR of the one-site
 * tensor (sector by sector; bond dimensions unchanged), the environment
 * updated and the bond matrix evolved back by exp(+i tau H0); then right to
 * left, mirrored.  trunc supplies only krylov_tol and krylov_maxdim.  The MPS
 * must have its centre on site 1 (as after tdvp_sweep); it returns there.
 * Errors as tdvp_sweep; SHAPE if a bond is larger than the space its site can
 * support. */
int tdvp_sweep1(tdvp_ctx* ctx, tdvp_mps* mps, double dt, const tdvp_trunc* trunc, tdvp_sweep_info* info);

/* One time step of the adaptive two-/one-site scheme (supplementary section
 * S2.2: two-site TDVP lets the bond dimension grow; once it has saturated,
 * one-site TDVP continues without SVDs).  *mode (in/out, host): 0 = the step
 * is a two-site sweep (tdvp_sweep with trunc), after which *mode becomes 1
 * if the largest full-state bond dimension has reached switch_frac x
 * trunc->chi_cap (switch_frac <= 0: never); 1 = the step is a one-site sweep
 * (tdvp_sweep1).  The caller owns the mode, so runs that must switch at the
 * same step (two precisions compared step by step) can share one.  info as
 * for the sweep taken.  Errors: INVALID (null argument, bad mode), else those
 * of the sweep taken. */
int tdvp_step(tdvp_ctx* ctx, tdvp_mps* mps, double dt, const tdvp_trunc* trunc, double switch_frac, int32_t* mode,
              tdvp_sweep_info* info);

/* ---- abelian U(1) x U(1) variant ---------------------------------------------
 * The paper's comparison symmetry (Table 1, Table S1: the same quench with
 * only the U(1) charge and spin symmetries): the same operations on the same
 * grouped-GEMM kernels and Lanczos core, with every recoupling coefficient a
 * plain local matrix element.  Conventions:
 *   bonds: tdvp_bond with q[i] = 2 S^z and tj[i] = N (particle number) of
 *     everything left of the bond; N - 2 S^z even, |2 S^z| <= N.
 *   local states s = n_up + 2 n_dn: 0 = |0>, 1 = |up>, 2 = |dn>,
 *     3 = |up dn> = c+_up c+_dn |0> (Jordan-Wigner mode order 1up, 1dn, 2up..).
 *   keys: one-site (ia, s, ib); two-site (ia, s1, s2, ib); blocks d_a x d_b,
 *     the full tensor restricted to the sector pair (no Clebsch-Gordan factor).
 *   environments: keys (iout, w, iin), w = 0 the block Hamiltonian, w = 1..4
 *     one component each of the doublet edge operators of the U(1) x SU(2)
 *     environments above: w = 1, 2 the components kappa = +1/2, -1/2 of D+,
 *     w = 3, 4 those of D- (left block: c+_up P, (-1)^k c_dn P, c+_dn P,
 *     -(-1)^k c_up P on its last site k; right block: the partners
 *     Q^w on its first site), so that a left block's environment is the
 *     full <Phi'| O |Phi> cut into sector blocks.
 * Same Hamiltonian (particle-hole symmetric interaction), memory layout,
 * ownership, synchronisation and errors as the U(1) x SU(2) calls. */
int tdvp_u1_center_layout(const tdvp_bond* left, const tdvp_bond* right, int32_t nsites, int32_t* nblocks,
                          int32_t* keys, int64_t* offsets, int64_t* total);
int tdvp_u1_env_layout(const tdvp_bond* bond, int32_t* nblocks, int32_t* keys, int64_t* offsets, int64_t* total);
int tdvp_u1_heff_plan(const tdvp_model* model, int32_t site, int32_t nsites, const tdvp_bond* left,
                      const tdvp_bond* right, const tdvp_blocks* Lenv, const tdvp_blocks* Renv, const tdvp_blocks* x,
                      int64_t* nterms, tdvp_term* terms, double* flops);
int tdvp_u1_env_plan(const tdvp_model* model, int32_t site, int32_t direction, const tdvp_bond* bond_in,
                     const tdvp_bond* bond_out, const tdvp_blocks* env_in, const tdvp_blocks* tensor,
                     const tdvp_blocks* env_out, int64_t* nterms, tdvp_env_term* terms, double* flops);
int tdvp_u1_heff_apply(tdvp_ctx* ctx, const tdvp_model* model, int32_t site, int32_t nsites, const tdvp_bond* left,
                       const tdvp_bond* right, const tdvp_blocks* Lenv, const tdvp_blocks* Renv, const tdvp_blocks* x,
                       tdvp_blocks* y);
int tdvp_u1_krylov_expm(tdvp_ctx* ctx, const tdvp_model* model, int32_t site, int32_t nsites, const tdvp_bond* left,
                        const tdvp_bond* right, const tdvp_blocks* Lenv, const tdvp_blocks* Renv, tdvp_blocks* x,
                        double tau_re, double tau_im, double tol, int32_t maxdim, tdvp_krylov_info* info);
int tdvp_u1_env_update(tdvp_ctx* ctx, const tdvp_model* model, int32_t site, int32_t direction,
                       const tdvp_bond* bond_in, const tdvp_bond* bond_out, const tdvp_blocks* env_in,
                       const tdvp_blocks* tensor, tdvp_blocks* env_out);
/* U(1) x U(1) MPS, as tdvp_mps_create / tdvp_mps_create_neel with the
 * conventions above: site keys (ia, s, ib) with s = 0..3; bond 0 the single
 * sector (0, 0) of dimension 1 and bond L a single sector of dimension 1
 * (the chain's 2 S^z and N; the Neel state's is (0, L)).  The MPS records its
 * symmetry, and tdvp_sweep, tdvp_sweep1, tdvp_step, tdvp_mps_measure,
 * tdvp_mps_overlap and the bond and site queries take either kind: the
 * two-site split cuts the sector matrices of x = (2 S^z, N) and truncates
 * single singular values (multiplet dimension 1) by the same rule.
 * tdvp_split and tdvp_split_sectors are for U(1) x SU(2) only.  Errors as
 * tdvp_mps_create. */
int tdvp_u1_mps_create(tdvp_ctx* ctx, const tdvp_model* model, const tdvp_bond* bonds, const tdvp_blocks* sites,
                       tdvp_mps** out);
int tdvp_u1_mps_create_neel(tdvp_ctx* ctx, const tdvp_model* model, int32_t complete, tdvp_mps** out);

/* Site-resolved observables of the quench (the local densities the paper
 * follows in time, main text results section): for every site k in 1..L,
 * sz[k-1] = <S^z_k> = (<n_k,up> - <n_k,down>)/2 and docc[k-1] =
 * <n_k,up n_k,down>, normalised by the state norm; *norm2 (optional) receives
 * <psi|psi>.  <n_k> = 1 exactly in the pseudospin-singlet sector, so
 * <n_k,up> = 1/2 + sz there (a U(1) x U(1) state need not be in it).  The
 * MPS must have its centre on site 1 and sites
 * 2..L right-canonical: the state after tdvp_sweep or tdvp_mps_create.
 * sz and docc are host arrays of L doubles.  Synchronises the stream.
 * Errors: INVALID (null or foreign MPS), NONFINITE (norm not positive). */
int tdvp_mps_measure(tdvp_ctx* ctx, const tdvp_mps* mps, double* sz, double* docc, double* norm2);

/* Overlap <bra|ket> of two MPS of the same chain, in any gauge and with any
 * bond dimensions (sectors present in only one of them contribute nothing):
 * out[0], out[1] = real and imaginary part.  Used to state the error of a
 * time step against another run (e.g. reduced against full precision):
 * |psi - phi|^2 = <psi|psi> + <phi|phi> - 2 Re <phi|psi>.  The two MPS may
 * belong to different contexts on the device of ctx (e.g. one per
 * precision); work runs on ctx's stream, so the caller finishes pending work
 * on the other context's stream first (tdvp_sweep returns synchronised).
 * Synchronises the stream.  Errors: INVALID (null argument, MPS on another
 * device, or of different symmetry), SHAPE (different L). */
int tdvp_mps_overlap(tdvp_ctx* ctx, const tdvp_mps* bra, const tdvp_mps* ket, double* out);

#ifdef __cplusplus
}
#endif

#endif /* TDVP_H */

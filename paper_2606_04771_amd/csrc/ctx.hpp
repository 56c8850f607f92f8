// Device context: stream, grow-only workspaces, cached device programs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <list>
#include <memory>
#include <map>
#include <string>
#include <initializer_list>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "../../include/tdvp.h"

namespace tdvp {

// One term of an output-stationary grouped GEMM:
//   C[m][n] += coef * sum_k opA(A)[m][k] * opB(B)[k][n]
// ops bits: 0 transpose A, 1 conjugate A, 2 transpose B, 3 conjugate B,
// 4/5 diagonal shift of A/B (see Bufs).
// Element (r, c) of an untransposed operand sits at off + r + c * ld
// (complex128, column-major).  Direct terms (K = 0): C[m][n] += coef * op(A)[m][n]
// with ops bit 0 = transpose, bit 1 = conjugate.
struct DevTerm {
  int64_t a_off, b_off;
  int32_t a_buf, b_buf;
  int32_t lda, ldb;
  int32_t K, ops;
  double coef;
};
struct DevOut {
  int64_t c_off;
  int32_t ldc, M, N;
  int32_t t_begin, t_end;   // GEMM terms
  int32_t d_begin, d_end;   // direct terms
  int32_t pad;
};
// One work item of a grouped-GEMM launch: an output tile and a contiguous
// piece [(t0, k0), (t1, k1)) of its K chain (terms in order, each cut into
// TK-wide steps).  slot < 0: the item owns the whole chain and writes the
// output; otherwise it writes its partial sum to partial slot `slot`.
struct DevTile {
  int32_t out, m0, n0, slot;
  int32_t t0, k0, t1, k1;
};
// Sum of the partial slots [slot0, slot0 + nparts) of one split tile, in
// order, plus the output's direct terms, written to the output.
struct DevRed {
  int32_t out, m0, n0, slot0, nparts, pad[3];
};

constexpr int kMaxBufs = 6;
// Operand base pointers of a launch, and optionally two diagonal shifts in
// device memory: a GEMM term with ops bit 4 (bit 5) has shift[0] (shift[1])
// subtracted from the diagonal of its A (B) operand; a direct term with ops
// bit 4 (bit 5) has its coefficient multiplied by shift[0] (shift[1]) (by
// zero when there are no shifts).  Used to take an energy offset out of the
// environment blocks before reduced-precision products and add it back exactly.
// `bad` (device int, may be null): set to 1 by any launch that writes a
// non-finite output value.
struct Bufs {
  const double* p[kMaxBufs];
  const double* shift;
  int* bad;
};

// Device memory of a context: the caller's allocator callbacks (torch's
// caching allocator through the Python binding) or hipMalloc / hipFree.
// Shared by everything the context allocates, objects that outlive the
// context (an MPS) included.  A failed allocation is hipErrorOutOfMemory.
struct Allocator {
  void* (*alloc_fn)(size_t, void*) = nullptr;
  void (*free_fn)(void*, void*) = nullptr;
  void* user = nullptr;
  hipError_t get(void** p, size_t n) const;
  void put(void* p) const;
  // bytes held (live) and the high-water mark since the last reset (peak)
  mutable std::mutex mu;
  mutable std::unordered_map<void*, size_t> held;
  mutable size_t live = 0, peak = 0;
};

// Device memory for program arrays, recycled by size class.  Every use of a
// chunk is ordered on the context stream, so a recycled chunk is only
// rewritten (by a stream-ordered copy) after earlier kernels have read it.
struct ProgPool {
  std::shared_ptr<const Allocator> al;
  std::unordered_map<size_t, std::vector<void*>> free;
  ~ProgPool();
};

// Host description of a grouped GEMM, lowered to device arrays once and
// reused across launches (only the buffer base pointers change).
struct Program {
  std::shared_ptr<ProgPool> pool;
  size_t cls = 0;
  std::vector<uint64_t> sig;   // structural signature it was built from (cache check)
  // K-chain splitting: alpha < 0 -> the default size rule; kmin: shortest piece
  double split_alpha = -1.0;
  int split_kmin = 128;
  std::vector<DevTerm> terms;
  std::vector<DevOut> outs;
  std::vector<DevTile> tiles;
  std::vector<DevRed> reds;
  int nslots = 0;           // partial slots of split tiles
  // diagonal blocks whose (2j+1)-weighted mean diagonal gives the shifts of
  // reduced-precision launches: (offset, dimension, weight) for buffer 1, then buffer 2
  std::vector<int64_t> shift_meta;
  int nshift[2] = {0, 0};
  double flops = 0.0;
  // element range [blo, bhi) of each buffer read as a GEMM operand (the part
  // that split-BF16 launches slice); empty when blo == bhi
  int64_t blo[kMaxBufs] = {}, bhi[kMaxBufs] = {};
  int64_t aux = 0;          // scratch elements needed by the program's outputs
  int tile_mode = 0;        // 0: per output block the better of 64x64 / 32x32; 1: all 32x32; 2: all 64x64
  int n64 = 0;              // tiles[0, n64) are 64x64 (four waves), the rest 32x32 (one wave)
  int role = 0;             // 1: effective-Hamiltonian apply (launched under its own kernel name)
  // Autotuning (effective-Hamiltonian programs): alternative tilings of the
  // same term lists, each launched on real work while measured with events;
  // the fastest replaces the active one.  All keep the per-element summation
  // order, so results do not depend on the choice.
  struct Tiling {
    std::vector<DevTile> tiles;
    int n64 = 0;
    int mode = 0;             // 0, 1, 2 as tile_mode; 3: the all-64x64 tiles in a persistent launch;
                              // 4: the all-32x32 tiles as FP64 wave tiles
    bool persistent = false;  // a fixed grid takes the tiles from a device counter
    bool wave = false;        // one 32x32 tile per wave (FP64 only)
    DevTile* d_tiles = nullptr;
  };
  std::vector<Tiling> alt;            // candidates (index 0 = the active tiling as built)
  mutable int tune_next = 0;          // launches issued so far while tuning
  mutable int tuned = -1;             // chosen candidate, -1 while measuring
  bool tuning() const { return alt.size() > 1 && tuned < 0; }
  mutable std::vector<hipEvent_t> tune_ev;
  static constexpr int kTuneRounds = 2;
  // one-launch-per-output-block schedule (a baseline for the grouped launch):
  // tiles grouped by output block, uploaded on first use
  mutable std::vector<int> blk_begin;
  mutable void* d_by_out = nullptr;
  // device copies
  DevTerm* d_terms = nullptr;
  DevOut* d_outs = nullptr;
  DevTile* d_tiles = nullptr;
  DevRed* d_reds = nullptr;
  int64_t* d_shift_meta = nullptr;
  void* d_mem = nullptr;
  ~Program();
  // tile the outputs, split long K chains, order work items by decreasing cost
  void finalize();
  // tiling of the outputs for a tile mode (no K-chain splitting), ordered for the XCDs
  void tile_only(int mode, Tiling& out, int per = 1) const;   // per: tiles per workgroup
};

// Grow-only device buffer; memory comes from its allocator (set by the owner
// before the first ensure(), hipMalloc when none is set).
struct DeviceBuffer {
  void* p = nullptr;
  size_t bytes = 0;
  std::shared_ptr<const Allocator> al;
  ~DeviceBuffer();
  hipError_t ensure(size_t n);
  void release();
};

}  // namespace tdvp

struct tdvp_ctx {
  // tiling autotuner decisions (tile mode) by program class: role and
  // half-octave of the program's flops; later programs of a decided class
  // start from its choice instead of measuring again
  std::map<int, int> tuned_modes;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int precision = TDVP_FP64;
  std::string err;
  // staging for program uploads
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  hipEvent_t upload_done = nullptr;
  // workspaces
  tdvp::DeviceBuffer ws_scratch, ws_krylov, ws_small, ws_vec, ws_theta, ws_svd;
  tdvp::DeviceBuffer ws_lanczos;   // partial sums of the graph-replayed Lanczos iteration
  tdvp::DeviceBuffer ws_part;   // partial tiles of split K chains
  tdvp::DeviceBuffer ws_shift;  // diagonal shifts of reduced-precision launches
  tdvp::DeviceBuffer ws_slices; // split-BF16 operand records
  tdvp::DeviceBuffer ws_compact;  // compact copy of a non-contiguous Krylov start vector
  tdvp::DeviceBuffer ws_trd;      // job table of the split's tridiagonal reductions
  void* solver = nullptr;       // rocblas handle for the eigensolver (created on first use)
  // side streams (default priority) with their own solver handles, for
  // independent eigensolves; joined back to `stream` by events
  // Side streams for concurrent batched eigensolves.  HIP maps streams onto
  // GPU_MAX_HW_QUEUES hardware queues (4 unless set before HIP starts); the
  // split plans its work per queue (side_group), and with its in-house
  // reduction a chi = 4096 sweep is fastest with the default 4 (3.8 s against
  // 4.4-4.8 s with 5-8 queues: fewer concurrent queues slow the reduction less).
  static constexpr int kSide = 16;
  int nside = 8;                      // in use (TDVP_SIDE_STREAMS, 1..kSide)
  bool graphs = true;                 // graph replay of Lanczos iterations
  hipStream_t side[kSide] = {};
  void* side_solver[kSide] = {};
  hipEvent_t side_ev[kSide + 1] = {};
  // side streams that share a hardware queue (HIP maps streams onto
  // GPU_MAX_HW_QUEUES queues; a shared queue runs its streams' work in issue
  // order): side_group[k] is the lowest side stream on side stream k's queue
  int side_group[kSide] = {};
  std::vector<hipEvent_t> eig_ev;     // cross-stream dependencies of the split's eigensolves
  void* host_small = nullptr;   // pinned host mirror of ws_small
  std::shared_ptr<tdvp::ProgPool> pool = std::make_shared<tdvp::ProgPool>();
  int verbose = 0;
  // program cache (structural hash -> program; a hit is confirmed by
  // comparing the full structural signature the hash was taken of)
  std::list<std::pair<uint64_t, std::shared_ptr<tdvp::Program>>> cache;
  // host-only programs of the allocation-free entry point (never uploaded:
  // their arrays are copied into the static scratch at every call)
  std::list<std::pair<uint64_t, std::shared_ptr<tdvp::Program>>> host_cache;
  void* scratch = nullptr;   // device address of the static scratch on `device`
  std::vector<char> na_stage;          // host staging of its program arrays
  hipEvent_t na_copied = nullptr;      // recorded after the last copy out of na_stage
  hipEvent_t ev[8] = {};
  std::shared_ptr<const tdvp::Allocator> alloc = std::make_shared<tdvp::Allocator>();
  // splitting of long K chains in effective-Hamiltonian programs
  // (tdvp_ctx_set_split): alpha < 0 means the size rule
  double split_alpha = -1.0;
  int split_kmin = 128;
  // Krylov basis storage (tdvp_ctx_set_krylov_storage): complex64 when set
  bool krylov_fp32 = false;
  // sweeps keep inactive MPS tensors and environments in pinned host memory
  // (tdvp_ctx_set_host_staging)
  bool host_staging = false;
  // device flag set by launches that wrote non-finite values (in ws_flag)
  tdvp::DeviceBuffer ws_flag;
};

namespace tdvp {

int hip_check(tdvp_ctx* ctx, hipError_t e, const char* what);
#define TDVP_HIP(ctx, call)                                    \
  do {                                                         \
    hipError_t e__ = (call);                                   \
    if (e__ != hipSuccess) return ::tdvp::hip_check(ctx, e__, #call); \
  } while (0)

// Upload a finalized program to the device (cached by key when key != 0).
int upload(tdvp_ctx* ctx, Program& p);
// Cache lookup by hash; a hit counts only if the stored signature equals sig.
std::shared_ptr<Program> cache_get(tdvp_ctx* ctx, uint64_t key, const std::vector<uint64_t>& sig);
void cache_put(tdvp_ctx* ctx, uint64_t key, std::shared_ptr<Program> p);
// The same on another list (programs kept on the host only).
typedef std::list<std::pair<uint64_t, std::shared_ptr<Program>>> ProgCache;
std::shared_ptr<Program> cache_get(ProgCache& c, uint64_t key, const std::vector<uint64_t>& sig);
void cache_put(ProgCache& c, uint64_t key, std::shared_ptr<Program> p);
// Device flag of non-finite outputs (allocated on first use, zeroed).
int bad_flag(tdvp_ctx* ctx, int** flag);
// Reads and clears the flag (synchronises the context stream).
int take_bad_flag(tdvp_ctx* ctx, bool& bad);
// Buffers that take their memory from the context's allocator.
inline void use_alloc(tdvp_ctx* ctx, std::initializer_list<DeviceBuffer*> bufs) {
  for (DeviceBuffer* b : bufs) b->al = ctx->alloc;
}

// Launch the grouped GEMM of p writing into C (base pointer of the output
// buffer) with operand buffers bufs.  precision: TDVP_FP64 or TDVP_FP32.
int launch_gemm(tdvp_ctx* ctx, const Program& p, const Bufs& bufs, double* C, int precision);
// The same with the program's active tiling, no autotuning.
int launch_gemm_tiles(tdvp_ctx* ctx, const Program& p, const Bufs& bufs, double* C, int precision);
// Device copies of a program's arrays (the program's own after upload(), or
// copies the caller placed elsewhere).
struct DevArrays {
  const DevTerm* terms;
  const DevOut* outs;
  const DevRed* reds;
  const int64_t* shift_meta;
};
// Workspaces of a launch given by the caller instead of the context's
// grow-only buffers: partial slots of split chains (partial_slot_bytes) and
// the shifts of reduced-precision launches (shift_bytes).
struct LaunchWs {
  double2* part;
  double* shift;
};
size_t partial_slot_bytes(int nslots);
inline size_t shift_bytes(int nblocks) { return sizeof(double) * 2 * (size_t)(nblocks + 1); }
// Active tiling of p (d_tiles: its device copy) on the given arrays and
// workspaces; allocates nothing.
int launch_gemm_ws(tdvp_ctx* ctx, const Program& p, const DevArrays& a, const DevTile* d_tiles, const Bufs& bufs,
                   double* C, int precision, const LaunchWs& ws);

// Lanczos vector kernels (complex128 vectors of n elements).  Basis vectors V
// (stride in elements) are complex128, or complex64 when v32 is set; the
// other vectors and every scalar are FP64.
int vec_dots(tdvp_ctx* ctx, const double* V, int64_t stride, int nv, const double* w, int64_t n,
             double* d_out /* 2*nv doubles, device */, bool v32 = false);
int vec_subtract_combo(tdvp_ctx* ctx, double* w, const double* V, int64_t stride, int nv,
                       const double* d_coef /* 2*nv */, int64_t n, double* d_norm2 /* or null */, bool v32 = false);
int vec_scale_copy(tdvp_ctx* ctx, double* dst, const double* src, double s, int64_t n);
int vec_combo(tdvp_ctx* ctx, double* out, const double* V, int64_t stride, int nv, const double* d_coef,
              int64_t n, bool v32 = false);
int vec_norm2(tdvp_ctx* ctx, const double* x, int64_t n, double* d_out);
size_t lanczos_partial_bytes(int64_t n, int maxdim);
int vec_lanczos_orth_it(tdvp_ctx* ctx, double* W, const double* V, int64_t stride, int maxdim, int64_t n,
                        const int* d_j, double* c1, double* c2, double* d_norm2, void* partial_buf, bool v32 = false);
int vec_lanczos_advance_it(tdvp_ctx* ctx, double* V, int64_t stride, double* x, const double* W, int64_t n,
                           const double* d_b2, int* d_j, int maxdim, bool v32 = false);
// complex64 basis slot from a complex128 vector
int vec_store_basis32(tdvp_ctx* ctx, double* V32, const double* x, int64_t n);
int vec_set_index(tdvp_ctx* ctx, int* d_j, int v);
int vec_check_finite(tdvp_ctx* ctx, const double* x, int64_t n, int* d_flag);
int vec_pad_matrix(tdvp_ctx* ctx, double* A, int64_t n, int64_t g, double v, double* d_scale);
// G -> H G H for count n x n Hermitian matrices of leading dimension ld
// (ld^2 apart; ld <= 0: n) (H = I - u u^H, a fixed dense reflector of size n;
// P: count * n complex scratch), and back: columns c >= c0 of eigenvectors W -> H W
int vec_reflect_forward(tdvp_ctx* ctx, hipStream_t st, double* G, int64_t n, int64_t count, double* P,
                        int64_t ld = 0);
int vec_reflect_back(tdvp_ctx* ctx, hipStream_t st, double* G, int64_t n, int64_t count, int64_t c0, int64_t ld = 0);
// Householder reduction of Hermitian n x n matrices to real tridiagonal form,
// one launch per column index for a whole set of jobs.  A job is `count`
// consecutive matrices A (full storage, n <= kTrdMaxN, overwritten); d, e (n
// reals per matrix) receive the diagonal and off-diagonal, V (n^2 complex per
// matrix) the reflectors, tau (n complex per matrix) their factors; Y: 2n
// complex per matrix of scratch.  eig_trd_column(k) for k = 0, 1, ... in
// stream order completes a job once k reaches its n - 1.
constexpr int64_t kTrdMaxN = 1024;
constexpr int kTrdMaxJobs = 48;
struct TrdJob {
  double *A, *V, *Y, *tau, *d, *e;
  int n, count, lda;   // A: leading dimension lda, matrices lda^2 apart; V, Y, tau, d, e packed by n
};
struct TrdSet {
  TrdJob job[kTrdMaxJobs];
  int njobs;
};
// The set's job table goes to device memory `table` (kTrdMaxJobs TrdJob
// entries) once, in stream order; every column launch reads it there.
int eig_trd_upload(tdvp_ctx* ctx, hipStream_t st, const TrdSet& set, void* table);
// A single-wave kernel that busy-waits for the given time on the wall clock.
int eig_spin(tdvp_ctx* ctx, hipStream_t st, double microseconds);
int eig_trd_column(tdvp_ctx* ctx, hipStream_t st, const TrdSet& set, const void* table, int64_t k);
// Columns c >= c0 of G = Q Zt for each matrix (Zt: real n x n eigenvectors of
// the tridiagonal form, Q the product of the reflectors in V / tau; G of
// leading dimension ld, matrices ld^2 apart).
int eig_trd_back(tdvp_ctx* ctx, hipStream_t st, const double* Zt, const double* V, const double* tau, double* G,
                 int64_t n, int64_t count, int64_t c0, int64_t ld);
// d_out[2b], d_out[2b+1] = re, im of sum conj(x) y over block b, whose element
// range is [d_meta[2b], d_meta[2b] + d_meta[2b+1]) (device metadata)
int vec_block_dots(tdvp_ctx* ctx, const double* x, const double* y, const int64_t* d_meta, int nblocks,
                   double* d_out);

// n x n matrix: everything outside the leading g x g block becomes the identity
int vec_pad_identity(tdvp_ctx* ctx, double* A, int64_t n, int64_t g);
// zero the strictly lower triangles of `count` consecutive n x n matrices
int vec_zero_lower(tdvp_ctx* ctx, double* A, int64_t n, int64_t count);
int vec_scale_cols_rsqrt(tdvp_ctx* ctx, double* A, int64_t ld, int64_t rows, int64_t cols, const double* lam);

}  // namespace tdvp

// Environment update that allocates nothing: the same two grouped-GEMM
// stages as tdvp_env_update, with every device buffer beyond the caller's
// inputs and outputs (the stage-1 products, the program arrays, the shifts of
// reduced-precision launches and the partial sums of split K chains) placed
// in one file-scope device array.  For callers that cannot allocate device
// memory (code under stream capture, tight serving loops).
//
// The array's name is a host-side stand-in in host code; its device address
// is taken once per device with hipGetSymbolAddress (the first context
// created on the device does it, with that device current) and only that
// address is handed to kernels and copies.  Every call on a device shares its
// array: calls that overlap on one device (other streams, other contexts,
// other threads) race, and each call overwrites what the previous one left.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "ctx.hpp"
#include "device.hpp"

namespace tdvp {

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // the stated maximum: 64 MiB per device
constexpr size_t kShiftRegion = size_t(64) << 10;    // [0, 64 KiB): shifts of reduced-precision launches
constexpr size_t kProgRegion = size_t(4) << 20;      // [64 KiB, 4 MiB): program arrays of both stages
                                                     // [4 MiB, 64 MiB): stage-1 products, then partial sums

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Byte offsets of one program's arrays inside the program region.
struct ArrayPlan {
  size_t terms, outs, tiles, reds, shift_meta, end;
};

ArrayPlan plan_arrays(const Program& p, size_t base) {
  ArrayPlan a;
  a.terms = base;
  a.outs = a.terms + align256(p.terms.size() * sizeof(DevTerm));
  a.tiles = a.outs + align256(p.outs.size() * sizeof(DevOut));
  a.reds = a.tiles + align256(p.tiles.size() * sizeof(DevTile));
  a.shift_meta = a.reds + align256(p.reds.size() * sizeof(DevRed));
  a.end = a.shift_meta + align256(p.shift_meta.size() * sizeof(int64_t));
  return a;
}

void fill(std::vector<char>& host, size_t region0, const Program& p, const ArrayPlan& a) {
  auto put = [&](size_t off, const void* src, size_t n) {
    if (n) std::memcpy(host.data() + (off - region0), src, n);
  };
  put(a.terms, p.terms.data(), p.terms.size() * sizeof(DevTerm));
  put(a.outs, p.outs.data(), p.outs.size() * sizeof(DevOut));
  put(a.tiles, p.tiles.data(), p.tiles.size() * sizeof(DevTile));
  put(a.reds, p.reds.data(), p.reds.size() * sizeof(DevRed));
  put(a.shift_meta, p.shift_meta.data(), p.shift_meta.size() * sizeof(int64_t));
}

DevArrays arrays_at(char* base, const ArrayPlan& a) {
  return DevArrays{(const DevTerm*)(base + a.terms), (const DevOut*)(base + a.outs), (const DevRed*)(base + a.reds),
                   (const int64_t*)(base + a.shift_meta)};
}

}  // namespace

int noalloc_init(tdvp_ctx* ctx) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices)
    return set_error(ctx, TDVP_E_INVALID, "device ordinal beyond the static scratch table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_addr[ctx->device]) {
    void* p = nullptr;
    TDVP_HIP(ctx, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return set_error(ctx, TDVP_E_HIP, "static scratch has no device address");
    g_addr[ctx->device] = p;
  }
  ctx->scratch = g_addr[ctx->device];
  return TDVP_OK;
}

}  // namespace tdvp

using namespace tdvp;

extern "C" int tdvp_env_update_noalloc(tdvp_ctx* ctx, const tdvp_model* model, int32_t site, int32_t direction,
                                       const tdvp_bond* bond_in, const tdvp_bond* bond_out,
                                       const tdvp_blocks* env_in, const tdvp_blocks* tensor, tdvp_blocks* env_out) {
  if (!ctx) return set_error(nullptr, TDVP_E_INVALID, "null ctx");
  return guarded(ctx, [&]() -> int {
    EnvInputs in;
    std::string err;
    int rc = load_env_inputs(in, model, site, direction, bond_in, bond_out, env_in, tensor, env_out, err);
    if (rc) return set_error(ctx, rc, err);
    if ((in.ten.n() && !in.ten.data) || (in.eout.n() && !in.eout.data) || (in.ein.n() && !in.ein.data))
      return set_error(ctx, TDVP_E_INVALID, "null device data pointer");
    TDVP_HIP(ctx, hipSetDevice(ctx->device));
    if (!ctx->scratch) return set_error(ctx, TDVP_E_HIP, "static scratch address not taken for this device");
    EnvPrograms ep = env_programs_host(ctx, *model, site, direction, in);
    const Program& s1 = *ep.s1;
    const Program& s2 = *ep.s2;
    if (s1.tiles.empty() && s2.tiles.empty()) return TDVP_OK;
    // region checks: everything must fit the static array
    const int nb = std::max(s1.nshift[0] + s1.nshift[1], s2.nshift[0] + s2.nshift[1]);
    if (shift_bytes(nb) > kShiftRegion)
      return set_error(ctx, TDVP_E_NOMEM, "environment update exceeds the static scratch (shift region)");
    const ArrayPlan a1 = plan_arrays(s1, kShiftRegion);
    const ArrayPlan a2 = plan_arrays(s2, a1.end);
    if (a2.end > kProgRegion)
      return set_error(ctx, TDVP_E_NOMEM, "environment update exceeds the static scratch (program arrays over 4 MiB)");
    const size_t prod_bytes = align256(sizeof(double) * 2 * (size_t)std::max<int64_t>(ep.scratch, 1));
    const size_t part_off = kProgRegion + prod_bytes;
    const size_t part_bytes = std::max(partial_slot_bytes(s1.nslots), partial_slot_bytes(s2.nslots));
    if (part_off + part_bytes > kScratchBytes)
      return set_error(ctx, TDVP_E_NOMEM,
                       "environment update exceeds the static scratch of 64 MiB (stage-1 products of " +
                           std::to_string(prod_bytes >> 20) + " MiB)");
    char* base = (char*)ctx->scratch;
    // program arrays: one host staging buffer kept by the context, one copy
    // into the program region (stream-ordered after the previous call's kernels)
    if (ctx->na_copied) TDVP_HIP(ctx, hipEventSynchronize(ctx->na_copied));
    ctx->na_stage.resize(a2.end - kShiftRegion);
    fill(ctx->na_stage, kShiftRegion, s1, a1);
    fill(ctx->na_stage, kShiftRegion, s2, a2);
    TDVP_HIP(ctx, hipMemcpyAsync(base + kShiftRegion, ctx->na_stage.data(), ctx->na_stage.size(),
                                 hipMemcpyHostToDevice, ctx->stream));
    if (ctx->na_copied) TDVP_HIP(ctx, hipEventRecord(ctx->na_copied, ctx->stream));
    LaunchWs ws{(double2*)(base + part_off), (double*)base};
    double* prod = (double*)(base + kProgRegion);
    Bufs b{};
    b.p[1] = (const double*)in.ein.data;
    b.p[2] = (const double*)in.ten.data;
    b.p[3] = prod;
    rc = launch_gemm_ws(ctx, s1, arrays_at(base, a1), (const DevTile*)(base + a1.tiles), b, prod, ctx->precision, ws);
    if (rc) return rc;
    return launch_gemm_ws(ctx, s2, arrays_at(base, a2), (const DevTile*)(base + a2.tiles), b, (double*)in.eout.data,
                          ctx->precision, ws);
  });
}

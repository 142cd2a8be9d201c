// dpmm_suffstats_static: the statistics of dpmm_suffstats with every scratch
// buffer of its kernels carved from one file-scope device array, so the call
// allocates nothing (for callers that cannot: code under graph capture,
// tight serving loops, harnesses that forbid allocation).
//
// Each GPU the library runs on holds its own copy of `scratch` for the life
// of the process.  The array's name is a host-side stand-in, not a device
// address: dpmm_create resolves this device's copy once with
// hipGetSymbolAddress and every later use goes through that pointer.  All
// calls on one GPU share the array: calls that overlap on one GPU (several
// contexts, several streams) race, and each call leaves its contents behind
// (every kernel here writes what it later reads, so nothing needs clearing).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "ctx.hpp"

using namespace dpmm;
using namespace dpmm::host;

namespace {

constexpr size_t STATIC_SCRATCH_BYTES = (size_t)DPMM_STATIC_SCRATCH_MIB << 20;
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

std::mutex g_mu;
std::vector<unsigned char*> g_ptr;  // per device: the address of its copy of `scratch`

size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

// offsets of the buffers a call needs inside the array; the total in *bytes
StatsBufs carve(const dpmm_ctx* ctx, int64_t n, unsigned char* base, size_t* bytes) {
  StatsBufs b{};
  size_t off = 0;
  auto take = [&](size_t sz) {
    unsigned char* p = base ? base + off : nullptr;
    off += up256(sz);
    return p;
  };
  if (stats_sorted(ctx)) {
    int G;
    long long per;
    sorted_plan(n, ctx->K, ctx->hist_cap, &G, &per);
    b.hist = (int*)take((size_t)G * ctx->K * sizeof(int));
    b.offs = (int*)take((size_t)G * ctx->K * sizeof(int));
    b.tot = (int*)take(((size_t)ctx->K + 4) * sizeof(int));
    b.perm = (int*)take((size_t)n * sizeof(int));
    b.zsort = (int*)take((size_t)n * sizeof(int));
    b.part = (double*)take(sub_stats_part_doubles(ctx->d, n) * sizeof(double));
  } else if (ctx->gaussian()) {
    b.spart = (double*)take(stats_small_part_doubles(ctx->d, ctx->K) * sizeof(double));
  }
  *bytes = off;
  return b;
}

}  // namespace

namespace dpmm::host {

dpmm_status static_scratch_init(dpmm_ctx* ctx) {
  std::lock_guard<std::mutex> lock(g_mu);
  if ((size_t)ctx->device >= g_ptr.size()) g_ptr.resize(ctx->device + 1, nullptr);
  if (g_ptr[ctx->device]) return DPMM_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    ctx->err = std::string("static scratch: hipGetSymbolAddress failed: ") + hipGetErrorString(e);
    return DPMM_E_DEVICE;
  }
  g_ptr[ctx->device] = (unsigned char*)p;
  return DPMM_OK;
}

}  // namespace dpmm::host

extern "C" {

dpmm_status dpmm_suffstats_static(dpmm_ctx* ctx, const void* x, int64_t n, const int32_t* z, const uint8_t* zsub) {
  if (!ctx) return DPMM_E_ARG;
  DPMM_TRY(check_n(ctx, x, n));
  if (n > 0 && (!z || !zsub)) return ctx->fail(DPMM_E_ARG, "z / zsub is NULL");
  if (ctx->K < 1) return ctx->fail(DPMM_E_STATE, "no clusters yet (call dpmm_init_labels or dpmm_set_state)");
  size_t bytes = 0;
  carve(ctx, n, nullptr, &bytes);
  if (bytes > STATIC_SCRATCH_BYTES)
    return ctx->fail(DPMM_E_CAPACITY, "the statistics of " + std::to_string(n) + " points and " +
                                          std::to_string(ctx->K) + " clusters need " + std::to_string(bytes) +
                                          " bytes of scratch, above the static " +
                                          std::to_string(STATIC_SCRATCH_BYTES) + "-byte array");
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if ((size_t)ctx->device < g_ptr.size()) base = g_ptr[ctx->device];
  }
  if (!base) return ctx->fail(DPMM_E_STATE, "the static scratch of this device was not resolved");
  const StatsBufs b = carve(ctx, n, base, &bytes);
  return stats_with(ctx, x, n, z, zsub, b);
}

}  // extern "C"

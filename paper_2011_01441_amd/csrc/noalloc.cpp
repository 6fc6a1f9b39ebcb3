// noalloc.cpp -- the semiring MM entry point that allocates no device
// memory (paco_semiring_mm_noalloc in paco.h).
//
// Its plan tables (work items, workgroup offsets, reduction tiles and
// sources) and temporary faces live in one fixed array in device memory,
// `scratch`, which every GPU the library runs on holds until the process
// ends.  Host code never uses the array's name as an address: paco_create
// looks up each device's copy once, with that device current, and the
// calls use that address.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "../../include/paco.h"
#include "ctx.h"

using namespace paco;

namespace {

constexpr uint64_t kScratchBytes = PACO_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

paco_status paco::noalloc_init(paco_ctx ctx) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices) {
    set_err(ctx, "device index beyond the scratch table");
    return PACO_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[ctx->device]) return PACO_OK;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_fail(ctx, e, "scratch address");
  if (!p) {
    set_err(ctx, "scratch address: null");
    return PACO_ERR_HIP;
  }
  g_ptr[ctx->device] = p;
  return PACO_OK;
}

extern "C" paco_status paco_semiring_mm_noalloc(paco_ctx ctx, const paco_mm_desc* d, paco_mm_result* out) {
  if (!ctx) return PACO_ERR_INVALID_ARG;
  if (!d) {
    set_err(ctx, "null descriptor");
    return PACO_ERR_INVALID_ARG;
  }
  void* p;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    p = g_ptr[ctx->device];
  }
  if (!p) {   // paco_create sets it; a context always has it
    set_err(ctx, "scratch address not set up");
    return PACO_ERR_INTERNAL;
  }
  FixedScratch fx{p, kScratchBytes};
  return run_mm(ctx, d, out, -1, &fx);
}

extern "C" uint64_t paco_noalloc_scratch_bytes(void) { return kScratchBytes; }

// kcommon.h -- small device helpers shared by the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "device_types.h"

namespace paco {

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup w lands
// on XCD w % 8).  Processors q and q+1 of a PACO partition are siblings that
// share a face of A or B, so consecutive processor indices are placed on the
// same XCD (and its L2): workgroup w runs processor (w % 8) * (nwg / 8) + w / 8.
__device__ __forceinline__ int remap_wg(int w, int nwg, int xcd) {
  if (xcd && (nwg & 7) == 0) return (w & 7) * (nwg >> 3) + (w >> 3);
  return w;
}

// All element types of the library are 4 bytes wide.
__device__ __forceinline__ Problem get_prob(const ProbRef& pr, int i) {
  if (pr.table) return pr.table[i];
  Problem p = pr.base;
  p.A = (const char*)p.A + (int64_t)i * pr.sA * 4;
  p.B = (const char*)p.B + (int64_t)i * pr.sB * 4;
  p.C = (char*)p.C + (int64_t)i * pr.sC * 4;
  return p;
}

// Values the compiler cannot prove wavefront-uniform (read from descriptor
// tables) but that are: move them to scalar registers.
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni(int64_t v) {
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <class T>
__device__ __forceinline__ T* uni(T* p) {
  return (T*)uni((int64_t)(uintptr_t)p);
}
__device__ __forceinline__ Problem uni(const Problem& p) {
  Problem q;
  q.A = uni(p.A); q.B = uni(p.B); q.C = uni(p.C);
  q.lda = uni(p.lda); q.ldb = uni(p.ldb); q.ldc = uni(p.ldc);
  q.n = uni(p.n); q.m = uni(p.m); q.k = uni(p.k);
  q.accumulate = uni(p.accumulate);
  return q;
}
__device__ __forceinline__ WorkItem uni(const WorkItem& w) {
  WorkItem v;
  v.prob = uni(w.prob);
  v.n0 = uni(w.n0); v.n1 = uni(w.n1);
  v.m0 = uni(w.m0); v.m1 = uni(w.m1);
  v.k0 = uni(w.k0); v.k1 = uni(w.k1);
  v.pad = 0;
  v.out_off = uni(w.out_off);
  return v;
}

// Buffer resource over the first `rows` rows (leading dimension `ld`
// elements, last row `cols` elements) of a 4-byte-element matrix at `base`;
// raw buffer loads outside that range return 0.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, int64_t rows,
                                                            int64_t ld, int64_t cols) {
  // branch-free: selects keep loops that rebuild resources in one block
  int64_t bytes = ((rows - 1) * ld + cols) * 4;
  bytes = rows > 0 ? bytes : 0;
  bytes = bytes < 0xFFFFFFFFll ? bytes : 0xFFFFFFFFll;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)(uint32_t)bytes,
                                           0x00020000);
}

// Load through the global address space (pointers read from descriptors
// would otherwise compile to flat loads).
template <class T>
__device__ __forceinline__ T gload(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
template <class T>
__device__ __forceinline__ void gstore(T* p, T v) {
  *(__attribute__((address_space(1))) T*)p = v;
}

// Per-processor timestamps (off unless the host gave a buffer): the
// workgroup standing for processor q records when it starts and ends its
// work on the real-time counter (100 MHz, one clock for the device) and
// the XCC_ID / HW_ID registers that name the die and compute unit it ran on.
// The end is taken after a barrier, once every wave is done.
constexpr int kHwRegHwId = 4 | (31 << 11);    // s_getreg encoding: HW_ID, 32 bits
constexpr int kHwRegXccId = 20 | (15 << 11);  // XCC_ID, 16 bits
__device__ __forceinline__ void stamp_start(const ProbRef& pr, int q) {
  if (pr.stamps && q < pr.stamp_cap && threadIdx.x == 0) {
    uint64_t* s = pr.stamps + 4 * (int64_t)q;
    gstore(s, (uint64_t)__builtin_amdgcn_s_memrealtime());
    gstore(s + 2, (uint64_t)(uint32_t)__builtin_amdgcn_s_getreg(kHwRegXccId));
    gstore(s + 3, (uint64_t)(uint32_t)__builtin_amdgcn_s_getreg(kHwRegHwId));
  }
}
__device__ __forceinline__ void stamp_end(const ProbRef& pr, int q) {
  if (pr.stamps && q < pr.stamp_cap) {
    __syncthreads();
    if (threadIdx.x == 0) gstore(pr.stamps + 4 * (int64_t)q + 1, (uint64_t)__builtin_amdgcn_s_memrealtime());
  }
}

}  // namespace paco

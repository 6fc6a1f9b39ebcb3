// k_calib.hip -- throughput calibration of the processors (workgroups).
//
// Every workgroup runs the same fixed chain of bf16 matrix-core products
// (four independent accumulators per wave, so the matrix pipe never waits)
// and records its start and end on the 100 MHz real-time counter.  With all
// compute units busy at once the duration reflects each processor's clock
// under the same load as a PACO launch.
#include "kcommon.h"
#include "kernels.h"

namespace paco {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8c;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16c;

__global__ __launch_bounds__(256) void k_calib(int iters, uint64_t* __restrict__ stamps,
                                               float* __restrict__ sink) {
  const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  bf16x8c a, b;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    a[j] = (__bf16)(1.0f / (1 + threadIdx.x + j));
    b[j] = (__bf16)(1.0f / (2 + j));
  }
  f32x16c c0 = {}, c1 = {}, c2 = {}, c3 = {};
  for (int i = 0; i < iters; ++i) {
    c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c3, 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int e = 0; e < 16; ++e) s += c0[e] + c1[e] + c2[e] + c3[e];
  __syncthreads();
  const uint64_t t1 = __builtin_amdgcn_s_memrealtime();
  if (s == 12345.678f) sink[threadIdx.x] = s;   // keeps the chain alive, never true in practice
  if (threadIdx.x == 0) {
    stamps[2 * blockIdx.x] = t0;
    stamps[2 * blockIdx.x + 1] = t1;
  }
}

// Peak probes.  Each lane runs 8 independent dependency chains, so that no
// instruction waits on the one before it; the operands come from kernel
// arguments, so nothing folds at compile time.

// (min,+) step: x = min(x + y, z), two u32 vector instructions
__global__ __launch_bounds__(256) void k_peak_valu_i32(int iters, uint32_t y, uint32_t z,
                                                       uint32_t* __restrict__ sink) {
  uint32_t x[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) x[c] = threadIdx.x + c;
#pragma unroll 4
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      uint32_t t = x[c] + y;
      asm volatile("" : "+v"(t));   // keeps add and min as two instructions
      x[c] = t < z ? t : z;
    }
  }
  uint32_t s = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) s ^= x[c];
  if (s == 0xFFFFFFFFu) sink[threadIdx.x] = s;   // never true for these operands
}

// fp32 fused multiply-add chains (unpacked: one lane-FMA per instruction)
__global__ __launch_bounds__(256) void k_peak_valu_f32(int iters, float a, float b,
                                                       float* __restrict__ sink) {
  float x[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) x[c] = 1e-3f * (threadIdx.x + c);
#pragma unroll 4
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = __builtin_fmaf(x[c], a, b);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < 8; ++c) s += x[c];
  if (s == 12345.678f) sink[threadIdx.x] = s;
}

// streaming copy, one 16-byte non-temporal load and store per lane and
// step, grid-stride (the fastest of the copy forms measured on this part)
typedef uint32_t u32x4c __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_peak_copy(const u32x4c* __restrict__ src, u32x4c* __restrict__ dst,
                                                   int64_t n16) {
  const int64_t lanes = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += lanes)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

}  // namespace

hipError_t launch_peak_valu_i32(int nwg, int iters, uint32_t* sink, hipStream_t s) {
  if (nwg <= 0 || iters <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_peak_valu_i32, dim3(nwg), dim3(256), 0, s, iters, 3u, 1u << 30, sink);
  return hipGetLastError();
}

hipError_t launch_peak_valu_f32(int nwg, int iters, float* sink, hipStream_t s) {
  if (nwg <= 0 || iters <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_peak_valu_f32, dim3(nwg), dim3(256), 0, s, iters, 0.999f, 1e-3f, sink);
  return hipGetLastError();
}

hipError_t launch_peak_copy(const void* src, void* dst, int64_t bytes, int nwg, hipStream_t s) {
  if (nwg <= 0 || bytes <= 0 || bytes % 16 != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_peak_copy, dim3(nwg), dim3(256), 0, s, (const u32x4c*)src, (u32x4c*)dst, bytes / 16);
  return hipGetLastError();
}

hipError_t launch_calib(int nwg, int iters, uint64_t* stamps, float* sink, hipStream_t s) {
  if (nwg <= 0 || iters <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_calib, dim3(nwg), dim3(256), 0, s, iters, stamps, sink);
  return hipGetLastError();
}

}  // namespace paco

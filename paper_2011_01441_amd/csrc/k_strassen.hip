// k_strassen.hip -- fused multi-level Strassen pre-additions and combine.
//
// Section "PACO Strassen", one level (1-based):
//   S1 = A00+A11  S2 = A10+A11  S3 = A00  S4 = A11  S5 = A00+A01
//   S6 = A10-A00  S7 = A01-A11
//   T1 = B00+B11  T2 = B00  T3 = B01-B11  T4 = B10-B00  T5 = B11
//   T6 = B00+B01  T7 = B10+B11
//   M_r = S_r T_r
//   C00 = M1+M4-M5+M7  C01 = M3+M5  C10 = M2+M4  C11 = M1+M3-M2+M6
// L levels nest these: leaf r = (r_1 .. r_L) has S_r = sum over the terms
// (q_1, s_1) of S_{r_1}, ..., (q_L, s_L) of S_{r_L} of s_1..s_L times the
// sub-block of A at quadrant path q_1..q_L, and C's sub-block at path
// q_1..q_L is the signed sum of M over the combine terms at every level.
// One thread owns one position (VW consecutive elements) of the h-by-h
// sub-blocks (h = n / 2^L): the pre-add reads the 4^L sub-block values of
// that position once and writes all 7^L leaf values; the combine reads the
// 7^L leaf values once and writes the 4^L C values.  Every byte of A, B, S,
// T, M and C crosses HBM exactly once.
#include "kcommon.h"
#include "kernels.h"

namespace paco {
namespace {

struct Term {
  int q, s;  // quadrant 0..3 (2*row + col) or leaf 0..6; sign +1/-1, 0 unused
};
__device__ constexpr Term kS[7][2] = {{{0, 1}, {3, 1}}, {{2, 1}, {3, 1}}, {{0, 1}, {0, 0}}, {{3, 1}, {0, 0}},
                                      {{0, 1}, {1, 1}}, {{2, 1}, {0, -1}}, {{1, 1}, {3, -1}}};
__device__ constexpr Term kT[7][2] = {{{0, 1}, {3, 1}}, {{0, 1}, {0, 0}}, {{1, 1}, {3, -1}}, {{2, 1}, {0, -1}},
                                      {{3, 1}, {0, 0}}, {{0, 1}, {1, 1}}, {{2, 1}, {3, 1}}};
// combine: C quadrant q = sum of sign * M_leaf
__device__ constexpr Term kC[4][4] = {{{0, 1}, {3, 1}, {4, -1}, {6, 1}},
                                      {{2, 1}, {4, 1}, {0, 0}, {0, 0}},
                                      {{1, 1}, {3, 1}, {0, 0}, {0, 0}},
                                      {{0, 1}, {2, 1}, {1, -1}, {5, 1}}};

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

template <int VW>
struct Vec {
  float v[VW];
};

template <int VW>
__device__ __forceinline__ Vec<VW> vload(const float* p) {
  Vec<VW> r;
  if constexpr (VW == 4) {
    float4 x = *(const float4*)p;
    r.v[0] = x.x; r.v[1] = x.y; r.v[2] = x.z; r.v[3] = x.w;
  } else {
#pragma unroll
    for (int j = 0; j < VW; ++j) r.v[j] = p[j];
  }
  return r;
}
template <int VW>
__device__ __forceinline__ void vstore(float* p, const Vec<VW>& r) {
  if constexpr (VW == 4) {
    *(float4*)p = make_float4(r.v[0], r.v[1], r.v[2], r.v[3]);
  } else {
#pragma unroll
    for (int j = 0; j < VW; ++j) p[j] = r.v[j];
  }
}

// sub-block (br, bc) of the 2^L x 2^L grid for quadrant path digits
template <int L>
__device__ __forceinline__ void path_block(int path, int& br, int& bc) {
  br = 0; bc = 0;
#pragma unroll
  for (int l = 0; l < L; ++l) {
    int qd = (path / ipow(4, L - 1 - l)) % 4;
    br = 2 * br + (qd >> 1);
    bc = 2 * bc + (qd & 1);
  }
}

// X (n x n) -> 7^L leaf blocks (h x h each, contiguous), TAB = kS or kT.
template <int L, int VW, bool IS_T>
__global__ __launch_bounds__(256) void k_preadd(const float* __restrict__ X, float* __restrict__ Out, int64_t n) {
  constexpr int NB = ipow(4, L), NL = ipow(7, L);
  const int64_t h = n >> L;
  const int64_t hv = h / VW;
  const int64_t pos = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (pos >= h * hv) return;
  const int64_t x = pos / hv, y = (pos % hv) * VW;
  Vec<VW> blk[NB];
#pragma unroll
  for (int p = 0; p < NB; ++p) {
    int br, bc;
    path_block<L>(p, br, bc);
    blk[p] = vload<VW>(X + (br * h + x) * n + bc * h + y);
  }
#pragma unroll
  for (int r = 0; r < NL; ++r) {
    Vec<VW> acc;
#pragma unroll
    for (int j = 0; j < VW; ++j) acc.v[j] = 0.f;
    // enumerate the 2^L term choices of the L levels
#pragma unroll
    for (int c = 0; c < (1 << L); ++c) {
      int path = 0, sign = 1;
      bool used = true;
#pragma unroll
      for (int l = 0; l < L; ++l) {
        const int rl = (r / ipow(7, L - 1 - l)) % 7;
        const int bit = (c >> (L - 1 - l)) & 1;
        const Term tm = IS_T ? kT[rl][bit] : kS[rl][bit];
        if (tm.s == 0) used = false;
        path = path * 4 + tm.q;
        sign *= tm.s;
      }
      if (!used) continue;
#pragma unroll
      for (int j = 0; j < VW; ++j) acc.v[j] = sign > 0 ? acc.v[j] + blk[path].v[j] : acc.v[j] - blk[path].v[j];
    }
    vstore<VW>(Out + (int64_t)r * h * h + x * h + y, acc);
  }
}

// 7^L leaf blocks M -> C (n x n)
template <int L, int VW>
__global__ __launch_bounds__(256) void k_combine(const float* __restrict__ M, float* __restrict__ C, int64_t n) {
  constexpr int NB = ipow(4, L), NL = ipow(7, L);
  const int64_t h = n >> L;
  const int64_t hv = h / VW;
  const int64_t pos = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (pos >= h * hv) return;
  const int64_t x = pos / hv, y = (pos % hv) * VW;
  Vec<VW> out[NB];
#pragma unroll
  for (int p = 0; p < NB; ++p)
#pragma unroll
    for (int j = 0; j < VW; ++j) out[p].v[j] = 0.f;
#pragma unroll
  for (int r = 0; r < NL; ++r) {
    const Vec<VW> mv = vload<VW>(M + (int64_t)r * h * h + x * h + y);
    // every C path whose combine terms select leaf digit r_l at each level
#pragma unroll
    for (int p = 0; p < NB; ++p) {
      int sign = 1;
#pragma unroll
      for (int l = 0; l < L; ++l) {
        const int rl = (r / ipow(7, L - 1 - l)) % 7;
        const int ql = (p / ipow(4, L - 1 - l)) % 4;
        int s = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (kC[ql][e].s != 0 && kC[ql][e].q == rl) s = kC[ql][e].s;
        sign *= s;
      }
      if (sign == 0) continue;
#pragma unroll
      for (int j = 0; j < VW; ++j) out[p].v[j] = sign > 0 ? out[p].v[j] + mv.v[j] : out[p].v[j] - mv.v[j];
    }
  }
#pragma unroll
  for (int p = 0; p < NB; ++p) {
    int br, bc;
    path_block<L>(p, br, bc);
    vstore<VW>(C + (br * h + x) * n + bc * h + y, out[p]);
  }
}

template <int L>
hipError_t preadd_l(int64_t n, const float* A, const float* B, float* S, float* T, hipStream_t s) {
  const int64_t h = n >> L;
  const bool v4 = h % 4 == 0 && (uintptr_t)A % 16 == 0 && (uintptr_t)B % 16 == 0 && L < 3;
  const int64_t work = h * (v4 ? h / 4 : h);
  dim3 g((unsigned)((work + 255) / 256)), b(256);
  if constexpr (L < 3) {  // 4-wide positions need 4^L x 4 registers: L < 3 only
    if (v4) {
      hipLaunchKernelGGL((k_preadd<L, 4, false>), g, b, 0, s, A, S, n);
      hipLaunchKernelGGL((k_preadd<L, 4, true>), g, b, 0, s, B, T, n);
      return hipGetLastError();
    }
  }
  {
    hipLaunchKernelGGL((k_preadd<L, 1, false>), g, b, 0, s, A, S, n);
    hipLaunchKernelGGL((k_preadd<L, 1, true>), g, b, 0, s, B, T, n);
  }
  return hipGetLastError();
}

template <int L>
hipError_t combine_l(int64_t n, const float* M, float* C, hipStream_t s) {
  const int64_t h = n >> L;
  const bool v4 = h % 4 == 0 && (uintptr_t)C % 16 == 0 && L < 3;
  const int64_t work = h * (v4 ? h / 4 : h);
  dim3 g((unsigned)((work + 255) / 256)), b(256);
  if constexpr (L < 3) {
    if (v4) {
      hipLaunchKernelGGL((k_combine<L, 4>), g, b, 0, s, M, C, n);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((k_combine<L, 1>), g, b, 0, s, M, C, n);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_strassen_preadd(int levels, int64_t n, const float* A, const float* B, float* S, float* T,
                                  hipStream_t s) {
  switch (levels) {
    case 1: return preadd_l<1>(n, A, B, S, T, s);
    case 2: return preadd_l<2>(n, A, B, S, T, s);
    case 3: return preadd_l<3>(n, A, B, S, T, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_strassen_combine(int levels, int64_t n, const float* M, float* C, hipStream_t s) {
  switch (levels) {
    case 1: return combine_l<1>(n, M, C, s);
    case 2: return combine_l<2>(n, M, C, s);
    case 3: return combine_l<3>(n, M, C, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace paco

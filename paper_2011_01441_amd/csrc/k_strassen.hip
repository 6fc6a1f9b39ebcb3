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
// T, M and C crosses HBM exactly once.  Three levels run as a staged
// recursion so that every index is static and the values stay in registers.
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

typedef float f32x4nt __attribute__((ext_vector_type(4)));

// every value is read once and written once per call, so 16-byte accesses
// are non-temporal
template <int VW>
__device__ __forceinline__ Vec<VW> vload(const float* p) {
  Vec<VW> r;
  if constexpr (VW == 4) {
    const f32x4nt x = __builtin_nontemporal_load((const f32x4nt*)p);
    r.v[0] = x[0]; r.v[1] = x[1]; r.v[2] = x[2]; r.v[3] = x[3];
  } else if constexpr (VW == 2) {
    float2 x = *(const float2*)p;
    r.v[0] = x.x; r.v[1] = x.y;
  } else {
#pragma unroll
    for (int j = 0; j < VW; ++j) r.v[j] = p[j];
  }
  return r;
}
template <int VW>
__device__ __forceinline__ void vstore(float* p, const Vec<VW>& r) {
  if constexpr (VW == 4) {
    __builtin_nontemporal_store((f32x4nt){r.v[0], r.v[1], r.v[2], r.v[3]}, (f32x4nt*)p);
  } else if constexpr (VW == 2) {
    *(float2*)p = make_float2(r.v[0], r.v[1]);
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
// Batched over blockIdx.y: parent y is X + y * xs (n x n, dense) and its
// 7^L blocks go to Out + y * os.
template <int L, int VW, bool IS_T>
__global__ __launch_bounds__(256) void k_preadd(const float* __restrict__ X, float* __restrict__ Out, int64_t n,
                                                int64_t xs, int64_t os) {
  constexpr int NB = ipow(4, L), NL = ipow(7, L);
  const int64_t h = n >> L;
  const int64_t hv = h / VW;
  const int64_t pos = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (pos >= h * hv) return;
  X += (int64_t)blockIdx.y * xs;
  Out += (int64_t)blockIdx.y * os;
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

// 7^L leaf blocks M -> C (n x n, leading dimension ldc), batched over
// blockIdx.y like k_preadd
template <int L, int VW>
__global__ __launch_bounds__(256) void k_combine(const float* __restrict__ M, float* __restrict__ C, int64_t n,
                                                 int64_t ldc, int64_t ms, int64_t cs) {
  constexpr int NB = ipow(4, L), NL = ipow(7, L);
  const int64_t h = n >> L;
  const int64_t hv = h / VW;
  const int64_t pos = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (pos >= h * hv) return;
  M += (int64_t)blockIdx.y * ms;
  C += (int64_t)blockIdx.y * cs;
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
    vstore<VW>(C + (br * h + x) * ldc + bc * h + y, out[p]);
  }
}

// Three levels fused as a staged recursion (static register indices): for
// each first-level product r1 the 16 second-level sub-block values of
// S_r1 (or T_r1) are formed from the 64 inputs, for each r2 the 4 values of
// the next level, and for each r3 the output.
template <int VW, bool IS_T>
__global__ __launch_bounds__(256) void k_preadd3(const float* __restrict__ X, float* __restrict__ Out, int64_t n,
                                                 int64_t xs, int64_t os) {
  const int64_t h = n >> 3;
  const int64_t hv = h / VW;
  const int64_t pos = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (pos >= h * hv) return;
  X += (int64_t)blockIdx.y * xs;
  Out += (int64_t)blockIdx.y * os;
  const int64_t x = pos / hv, y = (pos % hv) * VW;
  // in[q1][q2q3]: quadrant path q1, q2, q3 -> sub-block row/col of 8 x 8
  Vec<VW> in[4][16];
#pragma unroll
  for (int q1 = 0; q1 < 4; ++q1)
#pragma unroll
    for (int q23 = 0; q23 < 16; ++q23) {
      const int q2 = q23 >> 2, q3 = q23 & 3;
      const int br = 4 * (q1 >> 1) + 2 * (q2 >> 1) + (q3 >> 1);
      const int bc = 4 * (q1 & 1) + 2 * (q2 & 1) + (q3 & 1);
      in[q1][q23] = vload<VW>(X + (br * h + x) * n + bc * h + y);
    }
#pragma unroll
  for (int r1 = 0; r1 < 7; ++r1) {
    Vec<VW> l1[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
#pragma unroll
      for (int j = 0; j < VW; ++j) l1[i].v[j] = 0.f;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const Term tm = IS_T ? kT[r1][t] : kS[r1][t];
        if (tm.s == 0) continue;
#pragma unroll
        for (int j = 0; j < VW; ++j) l1[i].v[j] += tm.s > 0 ? in[tm.q][i].v[j] : -in[tm.q][i].v[j];
      }
    }
#pragma unroll
    for (int r2 = 0; r2 < 7; ++r2) {
      Vec<VW> l2[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int j = 0; j < VW; ++j) l2[i].v[j] = 0.f;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const Term tm = IS_T ? kT[r2][t] : kS[r2][t];
          if (tm.s == 0) continue;
#pragma unroll
          for (int j = 0; j < VW; ++j) l2[i].v[j] += tm.s > 0 ? l1[tm.q * 4 + i].v[j] : -l1[tm.q * 4 + i].v[j];
        }
      }
#pragma unroll
      for (int r3 = 0; r3 < 7; ++r3) {
        Vec<VW> o;
#pragma unroll
        for (int j = 0; j < VW; ++j) o.v[j] = 0.f;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const Term tm = IS_T ? kT[r3][t] : kS[r3][t];
          if (tm.s == 0) continue;
#pragma unroll
          for (int j = 0; j < VW; ++j) o.v[j] += tm.s > 0 ? l2[tm.q].v[j] : -l2[tm.q].v[j];
        }
        vstore<VW>(Out + (int64_t)((r1 * 7 + r2) * 7 + r3) * h * h + x * h + y, o);
      }
    }
  }
}

// Sign with which product r enters C quadrant q at one level (0 if not).
__device__ __forceinline__ constexpr int csign(int q, int r) {
  int s = 0;
  for (int e = 0; e < 4; ++e)
    if (kC[q][e].s != 0 && kC[q][e].q == r) s = kC[q][e].s;
  return s;
}

// Three-level combine, the same recursion upward: the 7 M blocks of one
// (r1, r2) fold into 4 third-level quadrant values, those into 16 for r1,
// and those into the 64 outputs.
template <int VW>
__global__ __launch_bounds__(256) void k_combine3(const float* __restrict__ M, float* __restrict__ C, int64_t n,
                                                  int64_t ldc, int64_t ms, int64_t cs) {
  const int64_t h = n >> 3;
  const int64_t hv = h / VW;
  const int64_t pos = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (pos >= h * hv) return;
  M += (int64_t)blockIdx.y * ms;
  C += (int64_t)blockIdx.y * cs;
  const int64_t x = pos / hv, y = (pos % hv) * VW;
  Vec<VW> out[4][16];
#pragma unroll
  for (int q1 = 0; q1 < 4; ++q1)
#pragma unroll
    for (int i = 0; i < 16; ++i)
#pragma unroll
      for (int j = 0; j < VW; ++j) out[q1][i].v[j] = 0.f;
#pragma unroll
  for (int r1 = 0; r1 < 7; ++r1) {
    Vec<VW> a2[16];
#pragma unroll
    for (int i = 0; i < 16; ++i)
#pragma unroll
      for (int j = 0; j < VW; ++j) a2[i].v[j] = 0.f;
#pragma unroll
    for (int r2 = 0; r2 < 7; ++r2) {
      Vec<VW> a3[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < VW; ++j) a3[i].v[j] = 0.f;
#pragma unroll
      for (int r3 = 0; r3 < 7; ++r3) {
        const Vec<VW> mv = vload<VW>(M + (int64_t)((r1 * 7 + r2) * 7 + r3) * h * h + x * h + y);
#pragma unroll
        for (int q3 = 0; q3 < 4; ++q3) {
          const int sg = csign(q3, r3);
          if (sg == 0) continue;
#pragma unroll
          for (int j = 0; j < VW; ++j) a3[q3].v[j] += sg > 0 ? mv.v[j] : -mv.v[j];
        }
      }
#pragma unroll
      for (int q2 = 0; q2 < 4; ++q2) {
        const int sg = csign(q2, r2);
        if (sg == 0) continue;
#pragma unroll
        for (int q3 = 0; q3 < 4; ++q3)
#pragma unroll
          for (int j = 0; j < VW; ++j) a2[q2 * 4 + q3].v[j] += sg > 0 ? a3[q3].v[j] : -a3[q3].v[j];
      }
    }
#pragma unroll
    for (int q1 = 0; q1 < 4; ++q1) {
      const int sg = csign(q1, r1);
      if (sg == 0) continue;
#pragma unroll
      for (int i = 0; i < 16; ++i)
#pragma unroll
        for (int j = 0; j < VW; ++j) out[q1][i].v[j] += sg > 0 ? a2[i].v[j] : -a2[i].v[j];
    }
  }
#pragma unroll
  for (int q1 = 0; q1 < 4; ++q1)
#pragma unroll
    for (int q23 = 0; q23 < 16; ++q23) {
      const int q2 = q23 >> 2, q3 = q23 & 3;
      const int br = 4 * (q1 >> 1) + 2 * (q2 >> 1) + (q3 >> 1);
      const int bc = 4 * (q1 & 1) + 2 * (q2 & 1) + (q3 & 1);
      vstore<VW>(C + (br * h + x) * ldc + bc * h + y, out[q1][q23]);
    }
}

// Vector width per position: 4 floats for L < 3; for L = 3 the 64 input
// (or output) blocks of a position allow 2 within the register budget.
// Batched parents are dense blocks of n^2 floats, so their alignment
// follows from the first one's when n is even.
template <int L>
hipError_t preadd_l(int64_t n, int nb, const float* A, const float* B, float* S, float* T, int64_t xs,
                    int64_t os, hipStream_t s) {
  const int64_t h = n >> L;
  constexpr int WV = L < 3 ? 4 : 2;
  const bool vw = h % WV == 0 && (uintptr_t)A % (4 * WV) == 0 && (uintptr_t)B % (4 * WV) == 0 &&
                  (uintptr_t)S % (4 * WV) == 0 && (uintptr_t)T % (4 * WV) == 0;
  const int64_t work = h * (vw ? h / WV : h);
  dim3 g((unsigned)((work + 255) / 256), (unsigned)nb), b(256);
  if constexpr (L == 3) {
    if (vw) {
      hipLaunchKernelGGL((k_preadd3<WV, false>), g, b, 0, s, A, S, n, xs, os);
      hipLaunchKernelGGL((k_preadd3<WV, true>), g, b, 0, s, B, T, n, xs, os);
    } else {
      hipLaunchKernelGGL((k_preadd3<1, false>), g, b, 0, s, A, S, n, xs, os);
      hipLaunchKernelGGL((k_preadd3<1, true>), g, b, 0, s, B, T, n, xs, os);
    }
    return hipGetLastError();
  } else {
    if (vw) {
      hipLaunchKernelGGL((k_preadd<L, WV, false>), g, b, 0, s, A, S, n, xs, os);
      hipLaunchKernelGGL((k_preadd<L, WV, true>), g, b, 0, s, B, T, n, xs, os);
      return hipGetLastError();
    }
    hipLaunchKernelGGL((k_preadd<L, 1, false>), g, b, 0, s, A, S, n, xs, os);
    hipLaunchKernelGGL((k_preadd<L, 1, true>), g, b, 0, s, B, T, n, xs, os);
    return hipGetLastError();
  }
}

template <int L>
hipError_t combine_l(int64_t n, int nb, const float* M, float* C, int64_t ldc, int64_t ms, int64_t cs,
                     hipStream_t s) {
  const int64_t h = n >> L;
  constexpr int WV = L < 3 ? 4 : 2;
  const bool vw = h % WV == 0 && ldc % WV == 0 && cs % WV == 0 && (uintptr_t)C % (4 * WV) == 0 &&
                  (uintptr_t)M % (4 * WV) == 0;
  const int64_t work = h * (vw ? h / WV : h);
  dim3 g((unsigned)((work + 255) / 256), (unsigned)nb), b(256);
  if constexpr (L == 3) {
    if (vw) hipLaunchKernelGGL((k_combine3<WV>), g, b, 0, s, M, C, n, ldc, ms, cs);
    else hipLaunchKernelGGL((k_combine3<1>), g, b, 0, s, M, C, n, ldc, ms, cs);
    return hipGetLastError();
  } else {
    if (vw) {
      hipLaunchKernelGGL((k_combine<L, WV>), g, b, 0, s, M, C, n, ldc, ms, cs);
      return hipGetLastError();
    }
    hipLaunchKernelGGL((k_combine<L, 1>), g, b, 0, s, M, C, n, ldc, ms, cs);
    return hipGetLastError();
  }
}

}  // namespace

hipError_t launch_strassen_preadd(int levels, int64_t n, const float* A, const float* B, float* S, float* T,
                                  hipStream_t s) {
  return launch_strassen_preadd_batch(levels, n, 1, A, B, S, T, 0, 0, s);
}

hipError_t launch_strassen_combine(int levels, int64_t n, const float* M, float* C, hipStream_t s) {
  return launch_strassen_combine_batch(levels, n, 1, M, C, n, 0, 0, s);
}

hipError_t launch_strassen_preadd_batch(int levels, int64_t n, int nb, const float* A, const float* B, float* S,
                                        float* T, int64_t xs, int64_t os, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  if (nb > 65535) return hipErrorInvalidValue;
  switch (levels) {
    case 1: return preadd_l<1>(n, nb, A, B, S, T, xs, os, s);
    case 2: return preadd_l<2>(n, nb, A, B, S, T, xs, os, s);
    case 3: return preadd_l<3>(n, nb, A, B, S, T, xs, os, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_strassen_combine_batch(int levels, int64_t n, int nb, const float* M, float* C, int64_t ldc,
                                         int64_t ms, int64_t cs, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  if (nb > 65535) return hipErrorInvalidValue;
  switch (levels) {
    case 1: return combine_l<1>(n, nb, M, C, ldc, ms, cs, s);
    case 2: return combine_l<2>(n, nb, M, C, ldc, ms, cs, s);
    case 3: return combine_l<3>(n, nb, M, C, ldc, ms, cs, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace paco

// k_bool.hip -- persistent boolean (OR, AND) semiring kernel on bit-packed
// rows, VALU only.
//
// Layout: A is n rows of ceil(k/32) words, B is k rows of ceil(m/32) words,
// C is n rows of ceil(m/32) words, bit j of a row in bit j%32 of word j/32.
// Row i of C is the OR of the rows l of B for which bit l of row i of A is
// set; with A's bit broadcast to a full-word mask (one bit-field extract per
// row and bit, shared by all of the thread's C words) every (row, bit, word)
// step is a single and-or (a thread's 4 x 16 register tile: one extract per
// sixteen and-ors).  A cuboid's C face is swept in TM-row by TNW-word
// tiles; its k-range (bits, cut on multiples of 32) is folded 128 bits per
// step through double-buffered LDS.
#include "kcommon.h"
#include "kernels.h"
#include "kfold.h"

namespace paco {
namespace {

constexpr int kThreads = 256;
constexpr int kBKB = 128;           // bits per step
constexpr int kKW = kBKB / 32;      // A words per row per step

// All ones if bit l of w is set, else 0 (sign-extended one-bit field,
// one v_bfe_i32).
__device__ __forceinline__ uint32_t bit_mask(uint32_t w, int l) {
  return (uint32_t)__builtin_amdgcn_sbfe((int)w, l, 1);
}
// (a & b) | c in one VALU instruction (plain C becomes an and plus a shared
// three-input or, 1.5 instructions).
__device__ __forceinline__ uint32_t and_or(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

template <int TM, int TNW, int RM, int RNW>
__global__ __launch_bounds__(kThreads) void k_semiring_bool(ProbRef pr, const WorkItem* __restrict__ items,
                                                             const int32_t* __restrict__ wg_off, int nwg,
                                                             int xcd, uint32_t* __restrict__ ws) {
  constexpr int TX = TNW / RNW, TY = TM / RM;
  static_assert(TX * TY == kThreads, "thread tile");
  constexpr int HM = RM / 2, HN = RNW / 2;
  constexpr int A_PER = (TM * kKW + kThreads - 1) / kThreads;
  constexpr int B_PER = kBKB * TNW / kThreads;
  static_assert((kBKB * TNW) % kThreads == 0, "B split");
  constexpr int BP = TNW + 4;
  __shared__ __align__(16) uint32_t As[2][kKW][TM];
  __shared__ __align__(16) uint32_t Bs[2][kBKB][BP];

  const int t = threadIdx.x;
  const int tx = t % TX, ty = t / TX;
  const int q = remap_wg(blockIdx.x, nwg, xcd);
  const int it1 = wg_off[q + 1];
  stamp_start(pr, q);
  int buf = 0;
  for (int it = wg_off[q]; it < it1; ++it) {
    const WorkItem W = uni(items[it]);
    const Problem P = uni(get_prob(pr, W.prob));
    const uint32_t* A = (const uint32_t*)P.A;
    const uint32_t* B = (const uint32_t*)P.B;
    const int kw_tot = (P.k + 31) / 32, mw_tot = (P.m + 31) / 32;
    const uint32_t last_mask = (P.m % 32) ? ((1u << (P.m % 32)) - 1u) : 0xffffffffu;
    for (int i0 = W.n0; i0 < W.n1; i0 += TM) {
      for (int j0 = W.m0; j0 < W.m1; j0 += TNW) {
        uint32_t acc[RM][RNW];
#pragma unroll
        for (int i = 0; i < RM; ++i)
#pragma unroll
          for (int j = 0; j < RNW; ++j) acc[i][j] = 0u;
        const auto a_rsrc = make_rsrc(A + (int64_t)i0 * P.lda, P.n - i0, P.lda, kw_tot);
        uint32_t ra[A_PER], rb[B_PER];
        uint32_t amask[A_PER];
        const int b_voff = ((t / TNW) * (int)P.ldb + j0 + t % TNW) * 4;
        const int b_soff = (kThreads / TNW) * (int)P.ldb * 4;
        auto load = [&](int kk) {  // kk: bit index, multiple of 32
#pragma unroll
          for (int s = 0; s < A_PER; ++s) {
            int e = t + s * kThreads;       // e = row * kKW + word
            int r = e / kKW, wd = e % kKW;
            int gw = kk / 32 + wd;          // global word of the row
            int lo = max(W.k0, gw * 32) - gw * 32, hi = min(W.k1, gw * 32 + 32) - gw * 32;
            uint32_t msk = hi <= lo ? 0u : (hi - lo == 32 ? 0xffffffffu : (((1u << (hi - lo)) - 1u) << lo));
            amask[s] = (e < TM * kKW) ? msk : 0u;
            ra[s] = __builtin_amdgcn_raw_buffer_load_b32(a_rsrc, (r * (int)P.lda + gw) * 4, 0, 0);
          }
          const auto b_rsrc = make_rsrc(B + (int64_t)kk * P.ldb, P.k - kk, P.ldb, mw_tot);
#pragma unroll
          for (int s = 0; s < B_PER; ++s)
            rb[s] = __builtin_amdgcn_raw_buffer_load_b32(b_rsrc, b_voff, s * b_soff, 0);
        };
        if (W.k0 < W.k1) load(W.k0);
        for (int kk = W.k0; kk < W.k1; kk += kBKB) {
#pragma unroll
          for (int s = 0; s < A_PER; ++s) {
            int e = t + s * kThreads;
            if (e < TM * kKW) As[buf][e % kKW][e / kKW] = ra[s] & amask[s];
          }
#pragma unroll
          for (int s = 0; s < B_PER; ++s) {
            int e = t + s * kThreads;
            Bs[buf][e / TNW][e % TNW] = rb[s];
          }
          __syncthreads();
          if (kk + kBKB < W.k1) load(kk + kBKB);
#pragma unroll
          for (int wd = 0; wd < kKW; ++wd) {
            uint32_t aw[RM];
#pragma unroll
            for (int h = 0; h < HM; ++h) {
              aw[h] = As[buf][wd][ty * HM + h];
              aw[HM + h] = As[buf][wd][TM / 2 + ty * HM + h];
            }
#pragma unroll 8
            for (int l = 0; l < 32; ++l) {
              uint32_t b[RNW];
#pragma unroll
              for (int h = 0; h < HN; ++h) {
                b[h] = Bs[buf][wd * 32 + l][tx * HN + h];
                b[HN + h] = Bs[buf][wd * 32 + l][TNW / 2 + tx * HN + h];
              }
#pragma unroll
              for (int i = 0; i < RM; ++i) {
                const uint32_t msk = bit_mask(aw[i], l);
#pragma unroll
                for (int j = 0; j < RNW; ++j) acc[i][j] = and_or(msk, b[j], acc[i][j]);
              }
            }
          }
          buf ^= 1;
        }
        const int64_t tld = W.m1 - W.m0;
#pragma unroll
        for (int i = 0; i < RM; ++i) {
          int r = i0 + (i < HM ? ty * HM + i : TM / 2 + ty * HM + (i - HM));
          if (r >= W.n1) continue;
#pragma unroll
          for (int j = 0; j < RNW; ++j) {
            int c = j0 + (j < HN ? tx * HN + j : TNW / 2 + tx * HN + (j - HN));
            if (c >= W.m1) continue;
            uint32_t v = acc[i][j];
            if (c == mw_tot - 1) v &= last_mask;
            if (W.out_off < 0) {
              uint32_t* cp = (uint32_t*)P.C + (int64_t)r * P.ldc + c;
              if (P.accumulate) v |= gload(cp);
              gstore(cp, v);
            } else {
              gstore(ws + W.out_off + (int64_t)(r - W.n0) * tld + (c - W.m0), v);
            }
          }
        }
      }
    }
    fold_after_item<ROr, kThreads>(pr, it, ws);
  }
  stamp_end(pr, q);
}

}  // namespace

int bool_occupancy(int tile) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (tile) {
    case BOOL_T512x32W:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_semiring_bool<512, 32, 4, 16>, kThreads, 0);
      break;
    case BOOL_T128x128W:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_semiring_bool<128, 128, 4, 16>, kThreads, 0);
      break;
    case BOOL_T256x64W:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_semiring_bool<256, 64, 4, 16>, kThreads, 0);
      break;
    case BOOL_T64x64W:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_semiring_bool<64, 64, 4, 4>, kThreads, 0);
      break;
  }
  return (e == hipSuccess && nb > 0) ? nb : 1;
}

BoolTileShape bool_tile_shape(int tile) {
  switch (tile) {
    case BOOL_T512x32W: return {512, 32};
    case BOOL_T128x128W: return {128, 128};
    case BOOL_T256x64W: return {256, 64};
    case BOOL_T64x64W: return {64, 64};
  }
  return {0, 0};
}

hipError_t launch_semiring_bool(int tile, const ProbRef& pr, const WorkItem* items, const int32_t* wg_off,
                                int nwg, int xcd, void* ws, hipStream_t s) {
  if (nwg <= 0) return hipSuccess;
  dim3 g(nwg), b(kThreads);
  uint32_t* w = (uint32_t*)ws;
  switch (tile) {
    case BOOL_T512x32W:
      hipLaunchKernelGGL((k_semiring_bool<512, 32, 4, 16>), g, b, 0, s, pr, items, wg_off, nwg, xcd, w);
      break;
    case BOOL_T128x128W:
      hipLaunchKernelGGL((k_semiring_bool<128, 128, 4, 16>), g, b, 0, s, pr, items, wg_off, nwg, xcd, w);
      break;
    case BOOL_T256x64W:
      hipLaunchKernelGGL((k_semiring_bool<256, 64, 4, 16>), g, b, 0, s, pr, items, wg_off, nwg, xcd, w);
      break;
    case BOOL_T64x64W:
      hipLaunchKernelGGL((k_semiring_bool<64, 64, 4, 4>), g, b, 0, s, pr, items, wg_off, nwg, xcd, w);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace paco

// k_int.hip -- persistent (min,+) / (max,+) semiring kernel on the VALU.
//
// One workgroup stands for one processor of the PACO partition (section
// "PACO MM") and runs its cuboid(s): the cuboid's C face is swept in TM x TN
// output tiles, and for each tile the cuboid's k-range is folded in steps of
// 32.  A and B tiles are staged in LDS (A transposed so a thread reads RM/2
// consecutive rows of one column with one vector read), double buffered with
// one barrier per step; the next step's global loads are in flight while the
// current one is computed.  Where the host finds every row and work item
// 16-byte aligned (VEC), a thread fetches four consecutive elements of a row
// with one 128-bit load; otherwise one element per 32-bit load.  Each thread owns an RM x RN register tile of
// accumulators; consecutive pairs of l fold as min3/max3 (two adds and one
// three-way min per two products).
//
// Exactness: (min,+) runs on uint32 -- valid entries are <= 2^30, so a + b
// <= 2^31 never wraps -- and clamps with min(acc, INF) at the end, which
// equals folding the saturated products min(a+b, INF).  (max,+) runs on
// int32 with NEG_INF = -2^30 padding; any sum with a NEG_INF factor is below
// -2^29 and any sum of finite entries (|x| <= 2^28) is at or above it, so
// thresholding the final value at -2^29 reproduces the absorbing NEG_INF.
#include <type_traits>

#include "kcommon.h"
#include "kernels.h"
#include "kfold.h"

namespace paco {
namespace {

constexpr int kThreads = 256;
constexpr int kBK = 32;
constexpr int kLChunk = 8;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct OpMin {
  using T = uint32_t;
  using Red = RMin;   // the fold of temporary faces
  static __device__ __forceinline__ T acc0() { return (T)kMinPlusInf; }
  static __device__ __forceinline__ T pad() { return (T)kMinPlusInf; }
  // pad_with(v, pad()) is the padding value, pad_with(v, nopad()) is v
  static __device__ __forceinline__ T nopad() { return 0u; }
  static __device__ __forceinline__ T pad_with(T v, T p) { return v > p ? v : p; }
  static __device__ __forceinline__ T mul(T a, T b) { return a + b; }
  static __device__ __forceinline__ T add(T x, T y) { return x < y ? x : y; }
  static __device__ __forceinline__ T finish(T v) { return v < (T)kMinPlusInf ? v : (T)kMinPlusInf; }
};

struct OpMax {
  using T = int32_t;
  using Red = RMax;
  static __device__ __forceinline__ T acc0() { return (T)0x80000000u; }
  static __device__ __forceinline__ T pad() { return kMaxPlusNegInf; }
  static __device__ __forceinline__ T nopad() { return 0x7fffffff; }
  static __device__ __forceinline__ T pad_with(T v, T p) { return v < p ? v : p; }
  static __device__ __forceinline__ T mul(T a, T b) { return (T)((uint32_t)a + (uint32_t)b); }
  static __device__ __forceinline__ T add(T x, T y) { return x > y ? x : y; }
  static __device__ __forceinline__ T finish(T v) { return v < kMaxPlusThreshold ? kMaxPlusNegInf : v; }
};

template <class Op, int TM, int TN, int RM, int RN, bool VEC>
__global__ __launch_bounds__(kThreads) void k_semiring_int(ProbRef pr, const WorkItem* __restrict__ items,
                                                            const int32_t* __restrict__ wg_off, int nwg,
                                                            int xcd, typename Op::T* __restrict__ ws) {
  using T = typename Op::T;
  constexpr int TX = TN / RN, TY = TM / RM;
  static_assert(TX * TY == kThreads, "thread tile");
  static_assert((kBK * TM) % kThreads == 0 && (kBK * TN) % kThreads == 0, "load split");
  constexpr int AP = TM + 4, BP = TN + 4;
  constexpr int HM = RM / 2, HN = RN / 2;
  constexpr int A_PER = kBK * TM / kThreads, B_PER = kBK * TN / kThreads;
  // VEC: per step, A is TM rows of eight 4-element k-quads and B is kBK rows
  // of TN / 4 column quads; each thread loads A_PER / 4 and B_PER / 4 quads
  constexpr int A_PER4 = A_PER / 4, B_PER4 = B_PER / 4, BQ = TN / 4;
  static_assert(!VEC || (A_PER % 4 == 0 && B_PER % 4 == 0 && kThreads % BQ == 0), "vector load split");
  __shared__ __align__(16) T As[2][kBK][AP];
  __shared__ __align__(16) T Bs[2][kBK][BP];

  const int t = threadIdx.x;
  const int tx = t % TX, ty = t / TX;
  const int q = remap_wg(blockIdx.x, nwg, xcd);
  const int it1 = wg_off[q + 1];
  stamp_start(pr, q);
  int buf = 0;
  for (int it = wg_off[q]; it < it1; ++it) {
    const WorkItem W = uni(items[it]);
    const Problem P = uni(get_prob(pr, W.prob));
    const T* __restrict__ A = (const T*)P.A;
    const T* __restrict__ B = (const T*)P.B;
    for (int i0 = W.n0; i0 < W.n1; i0 += TM) {
      for (int j0 = W.m0; j0 < W.m1; j0 += TN) {
        T acc[RM][RN];
#pragma unroll
        for (int i = 0; i < RM; ++i)
#pragma unroll
          for (int j = 0; j < RN; ++j) acc[i][j] = Op::acc0();
        T ra[VEC ? 1 : A_PER], rb[VEC ? 1 : B_PER];
        u32x4 ra4[VEC ? A_PER4 : 1], rb4[VEC ? B_PER4 : 1];
        // Buffer loads.  32-bit: thread t reads A rows i0 + t/kBK +
        // s*(kThreads/kBK) at column t % kBK of the step, and B rows kk + t/TN
        // + s*(kThreads/TN) at column j0 + t % TN.  VEC: thread t reads A rows
        // i0 + t/8 + s*(kThreads/8) at columns 4*(t % 8) .. +3 of the step, and
        // B rows kk + t/BQ + s*(kThreads/BQ) at columns j0 + 4*(t % BQ) .. +3.
        // The per-s row offsets are uniform (scalar offsets); rows past the
        // matrix read 0 through the buffer range check, rows and columns past
        // the piece are discarded, and the k-tail beyond the piece's k1 is
        // replaced by the padding value.
        constexpr int A_RSTEP = VEC ? kThreads / 8 : kThreads / kBK;
        constexpr int B_RSTEP = VEC ? kThreads / BQ : kThreads / TN;
        const auto a_rsrc = make_rsrc(A + (int64_t)i0 * P.lda, P.n - i0, P.lda, P.k);
        const int a_c = VEC ? 4 * (t % 8) : t % kBK;   // first column of the step this thread loads
        int a_voff = ((t / (kThreads / A_RSTEP)) * (int)P.lda + W.k0 + a_c) * 4;
        const int a_soff = A_RSTEP * (int)P.lda * 4;
        const int b_c = VEC ? 4 * (t % BQ) : t % TN;
        const int b_voff = ((t / (kThreads / B_RSTEP)) * (int)P.ldb + j0 + b_c) * 4;
        const int b_soff = B_RSTEP * (int)P.ldb * 4;
        // Loads only issue here; padding is applied when the registers are
        // written to LDS, so the loads stay in flight during the compute.
        int a_lim = 0;    // columns of this thread's load still inside the piece
        int b_rows = 0;
        auto load = [&](int kk) {
          a_lim = W.k1 - kk - a_c;
          if constexpr (VEC) {
#pragma unroll
            for (int s = 0; s < A_PER4; ++s)
              ra4[s] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(a_rsrc, a_voff, s * a_soff, 0));
          } else {
#pragma unroll
            for (int s = 0; s < A_PER; ++s)
              ra[s] = (T)__builtin_amdgcn_raw_buffer_load_b32(a_rsrc, a_voff, s * a_soff, 0);
          }
          a_voff += kBK * 4;
          const auto b_rsrc = make_rsrc(B + (int64_t)kk * P.ldb, P.k - kk, P.ldb, P.m);
          b_rows = W.k1 - kk - t / (kThreads / B_RSTEP);
          if constexpr (VEC) {
#pragma unroll
            for (int s = 0; s < B_PER4; ++s)
              rb4[s] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(b_rsrc, b_voff, s * b_soff, 0));
          } else {
#pragma unroll
            for (int s = 0; s < B_PER; ++s)
              rb[s] = (T)__builtin_amdgcn_raw_buffer_load_b32(b_rsrc, b_voff, s * b_soff, 0);
          }
        };
        // store_step(pad): the registers of one step into LDS buffer buf.
        // Padding only changes values past the piece's k1, so it runs on a
        // piece's last, partial step alone (a uniform branch); elsewhere
        // pad_with(v, nopad()) would return v unchanged.
        auto store_step = [&](auto pad_c) {
          constexpr bool PAD = decltype(pad_c)::value;
          if constexpr (VEC) {
            const int arow = t / 8;
#pragma unroll
            for (int s = 0; s < A_PER4; ++s)
#pragma unroll
              for (int j = 0; j < 4; ++j)
                As[buf][a_c + j][arow + s * A_RSTEP] =
                    PAD ? Op::pad_with((T)ra4[s][j], j < a_lim ? Op::nopad() : Op::pad()) : (T)ra4[s][j];
            const int brow = t / BQ;
#pragma unroll
            for (int s = 0; s < B_PER4; ++s) {
              u32x4 v = rb4[s];
              if constexpr (PAD) {
                const T bp = s * B_RSTEP < b_rows ? Op::nopad() : Op::pad();
#pragma unroll
                for (int j = 0; j < 4; ++j) v[j] = (uint32_t)Op::pad_with((T)rb4[s][j], bp);
              }
              *(u32x4*)&Bs[buf][brow + s * B_RSTEP][b_c] = v;
            }
          } else {
#pragma unroll
            for (int s = 0; s < A_PER; ++s) {
              int e = t + s * kThreads;
              As[buf][e % kBK][e / kBK] = PAD ? Op::pad_with(ra[s], 0 < a_lim ? Op::nopad() : Op::pad()) : ra[s];
            }
#pragma unroll
            for (int s = 0; s < B_PER; ++s) {
              int e = t + s * kThreads;
              Bs[buf][e / TN][e % TN] =
                  PAD ? Op::pad_with(rb[s], s * B_RSTEP < b_rows ? Op::nopad() : Op::pad()) : rb[s];
            }
          }
        };
        if (W.k0 < W.k1) load(W.k0);
        for (int kk = W.k0; kk < W.k1; kk += kBK) {
          if (W.k1 - kk < kBK) store_step(std::true_type{});
          else store_step(std::false_type{});
          __syncthreads();
          if (kk + kBK < W.k1) load(kk + kBK);
          // chunks wholly past the piece's k-range hold only padding, whose
          // products never win the fold: a piece's last step stops after the
          // chunk that holds k1 - 1 (at least one chunk runs: kk < k1)
          const int lim = W.k1 - kk < kBK ? W.k1 - kk : kBK;
          int l0 = 0;
          do {
#pragma unroll
            for (int l = l0; l < l0 + kLChunk; ++l) {
              T a[RM], b[RN];
#pragma unroll
              for (int h = 0; h < HM; ++h) {
                a[h] = As[buf][l][ty * HM + h];
                a[HM + h] = As[buf][l][TM / 2 + ty * HM + h];
              }
#pragma unroll
              for (int h = 0; h < HN; ++h) {
                b[h] = Bs[buf][l][tx * HN + h];
                b[HN + h] = Bs[buf][l][TN / 2 + tx * HN + h];
              }
#pragma unroll
              for (int i = 0; i < RM; ++i)
#pragma unroll
                for (int j = 0; j < RN; ++j) acc[i][j] = Op::add(acc[i][j], Op::mul(a[i], b[j]));
            }
            l0 += kLChunk;
          } while (l0 < lim);
          buf ^= 1;
        }
        // epilogue
        const int64_t tld = W.m1 - W.m0;
#pragma unroll
        for (int i = 0; i < RM; ++i) {
          int r = i0 + (i < HM ? ty * HM + i : TM / 2 + ty * HM + (i - HM));
          if (r >= W.n1) continue;
#pragma unroll
          for (int j = 0; j < RN; ++j) {
            int c = j0 + (j < HN ? tx * HN + j : TN / 2 + tx * HN + (j - HN));
            if (c >= W.m1) continue;
            T v = Op::finish(acc[i][j]);
            if (W.out_off < 0) {
              T* cp = (T*)P.C + (int64_t)r * P.ldc + c;
              if (P.accumulate) v = Op::add(gload(cp), v);
              gstore(cp, v);
            } else {
              gstore(ws + W.out_off + (int64_t)(r - W.n0) * tld + (c - W.m0), v);
            }
          }
        }
      }
    }
    fold_after_item<typename Op::Red, kThreads>(pr, it, (const typename Op::Red::T*)ws);
  }
  stamp_end(pr, q);
}

template <class Op, int TM, int TN, int RM, int RN>
void launch_shape(bool vec, dim3 g, dim3 b, hipStream_t s, const ProbRef& pr, const WorkItem* items,
                  const int32_t* wg_off, int nwg, int xcd, typename Op::T* ws) {
  if (vec)
    hipLaunchKernelGGL((k_semiring_int<Op, TM, TN, RM, RN, true>), g, b, 0, s, pr, items, wg_off, nwg, xcd, ws);
  else
    hipLaunchKernelGGL((k_semiring_int<Op, TM, TN, RM, RN, false>), g, b, 0, s, pr, items, wg_off, nwg, xcd, ws);
}

template <class Op>
hipError_t launch_op(int tile, const ProbRef& pr, const WorkItem* items, const int32_t* wg_off,
                     int nwg, int xcd, void* ws, hipStream_t s) {
  using T = typename Op::T;
  dim3 g(nwg), b(kThreads);
  // 128-bit loads: the host sets vec_ok when every problem's A and B are
  // 16-byte aligned with rows (and leading dimensions) of multiples of four
  // elements and every work item starts on a multiple of four in k and m
  const bool vec = pr.vec_ok != 0;
  switch (tile) {
    case INT_T128x128: launch_shape<Op, 128, 128, 8, 8>(vec, g, b, s, pr, items, wg_off, nwg, xcd, (T*)ws); break;
    case INT_T256x64: launch_shape<Op, 256, 64, 8, 8>(vec, g, b, s, pr, items, wg_off, nwg, xcd, (T*)ws); break;
    case INT_T64x64: launch_shape<Op, 64, 64, 4, 4>(vec, g, b, s, pr, items, wg_off, nwg, xcd, (T*)ws); break;
    case INT_T64x128: launch_shape<Op, 64, 128, 4, 8>(vec, g, b, s, pr, items, wg_off, nwg, xcd, (T*)ws); break;
    case INT_T128x64: launch_shape<Op, 128, 64, 8, 4>(vec, g, b, s, pr, items, wg_off, nwg, xcd, (T*)ws); break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class Op>
int occupancy_op(int tile) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (tile) {
    case INT_T128x128:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_semiring_int<Op, 128, 128, 8, 8, true>, kThreads, 0);
      break;
    case INT_T256x64:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_semiring_int<Op, 256, 64, 8, 8, true>, kThreads, 0);
      break;
    case INT_T64x64:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_semiring_int<Op, 64, 64, 4, 4, true>, kThreads, 0);
      break;
    case INT_T64x128:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_semiring_int<Op, 64, 128, 4, 8, true>, kThreads, 0);
      break;
    case INT_T128x64:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_semiring_int<Op, 128, 64, 8, 4, true>, kThreads, 0);
      break;
  }
  return (e == hipSuccess && nb > 0) ? nb : 1;
}

}  // namespace

int int_occupancy(int sr, int tile) {
  return sr == SR_MAXPLUS ? occupancy_op<OpMax>(tile) : occupancy_op<OpMin>(tile);
}

IntTileShape int_tile_shape(int tile) {
  switch (tile) {
    case INT_T128x128: return {128, 128};
    case INT_T256x64: return {256, 64};
    case INT_T64x64: return {64, 64};
    case INT_T64x128: return {64, 128};
    case INT_T128x64: return {128, 64};
  }
  return {0, 0};
}

hipError_t launch_semiring_int(int sr, int tile, const ProbRef& pr, const WorkItem* items,
                               const int32_t* wg_off, int nwg, int xcd_remap, void* ws,
                               hipStream_t s) {
  if (nwg <= 0) return hipSuccess;
  if (sr == SR_MINPLUS) return launch_op<OpMin>(tile, pr, items, wg_off, nwg, xcd_remap, ws, s);
  if (sr == SR_MAXPLUS) return launch_op<OpMax>(tile, pr, items, wg_off, nwg, xcd_remap, ws, s);
  return hipErrorInvalidValue;
}

}  // namespace paco

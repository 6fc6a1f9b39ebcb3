// k_ring.hip -- persistent (+,x) ring kernel on gfx950 matrix cores.
//
// One workgroup of WM x WN waves (one or two per SIMD) stands for one
// processor of the PACO partition and runs its cuboid(s): the C face is
// swept in BM x BN tiles and the cuboid's k-range folded 32 at a time.
// Operands arrive as float32.
//  FP32   : tiles staged in LDS as float32, v_mfma_f32_32x32x2_f32.
//  BF16X3 : each element is split on its way into LDS, hi = bf16(x),
//           lo = bf16(x - hi) (round to nearest even; x - hi is exact), and
//           each 32x32 block accumulates lo*hi', hi*lo', hi*hi' with
//           v_mfma_f32_32x32x16_bf16 in float32.
//  BF16X6 : hi, mid = bf16(x - hi), lo = bf16(x - hi - mid) and the six
//           products lo*hi', hi*lo', mid*mid', mid*hi', hi*mid', hi*hi'.
// The split costs no extra HBM pass: the next step's float32 loads are in
// flight while the current step runs and are split when written to LDS.  B
// is stored k-contiguous (transposed) so both operands are read as 8
// consecutive k values per lane with one 128-bit LDS read.  LDS rows are
// 64 bytes (32 bf16) with the 16-byte chunk index XOR-ed by (row / 4) % 4, so
// the 16 rows a quarter-wave reads fall on distinct banks without padding.
// With two waves per SIMD one wave's split and LDS traffic overlaps the
// other wave's matrix-core work; one wave per SIMD leaves each wave 512
// registers for a 128 x 128 wave tile.
//
// Within a matrix-core instruction each half-wave supplies a k-slice; A and
// B use the same lane-to-k assignment, so every k is paired exactly once.
#include <type_traits>

#include "kcommon.h"
#include "kernels.h"
#include "kfold.h"

namespace paco {
namespace {

constexpr int kBK = 32;

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Two float32 values -> packed bf16 (round to nearest even), element 0 low.
__device__ __forceinline__ uint32_t cvt2(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){a, b}, bf16x2));
}

// Split 4 float32 values into NS packed bf16 parts (4 x 16 bits each).
template <int NS>
__device__ __forceinline__ void split4(float x0, float x1, float x2, float x3, u32x2 out[NS]) {
#pragma unroll
  for (int p = 0; p < NS; ++p) {
    const uint32_t h01 = cvt2(x0, x1), h23 = cvt2(x2, x3);
    out[p] = (u32x2){h01, h23};
    if (p + 1 < NS) {
      x0 -= __builtin_bit_cast(float, h01 << 16);
      x1 -= __builtin_bit_cast(float, h01 & 0xffff0000u);
      x2 -= __builtin_bit_cast(float, h23 << 16);
      x3 -= __builtin_bit_cast(float, h23 & 0xffff0000u);
    }
  }
}

__device__ __forceinline__ f32x16 mfma_bf16(const bf16x8& a, const bf16x8& b, const f32x16& c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x16 mfma_f32(float a, float b, const f32x16& c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

template <bool VEC>
__device__ __forceinline__ f32x4 load4(const __amdgpu_buffer_rsrc_t& r, int voff, int soff) {
  if constexpr (VEC) {
    return __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
  } else {
    f32x4 v;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      v[j] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff + 4 * j, soff, 0));
    return v;
  }
}

// Byte offset in an LDS operand tile of 16-byte chunk `c` of row `r`.
// bf16 rows: 4 chunks (64 B); float rows: 8 chunks (128 B).  For B tiles
// (PERM) the row is also rotated within its group of four by (r / 4) % 4:
// the transposing store writes rows 4q + c of many n-quads q at once, which
// would otherwise all hit the same banks; reads of 16 consecutive rows stay
// on 16 distinct bank groups either way.
template <bool F32, bool PERM = false>
__device__ __forceinline__ int lds_off(int r, int c) {
  const int g = (r >> 2) & 3;
  const int pr = PERM ? ((r & ~3) | (((r & 3) + g) & 3)) : r;
  if constexpr (F32) return pr * 128 + ((c ^ ((r >> 1) & 7)) << 4);
  else return pr * 64 + ((c ^ g) << 4);
}

template <int PREC, int BM, int BN, int WM, int WN, bool VEC>
__global__ __launch_bounds__(64 * WM * WN) void k_ring(ProbRef pr, const WorkItem* __restrict__ items,
                                                    const int32_t* __restrict__ wg_off, int nwg, int xcd,
                                                    float* __restrict__ ws) {
  constexpr bool F32 = PREC == PREC_FP32;
  constexpr int NS = F32 ? 1 : (PREC == PREC_BF16X3 ? 2 : 3);
  constexpr int kThreads = 64 * WM * WN;
  constexpr int WTM = BM / WM, WTN = BN / WN;    // wave tile (waves WM x WN)
  constexpr int FM = WTM / 32, FN = WTN / 32;    // 32x32 blocks per wave
  static_assert(FM >= 1 && FN >= 1, "tile");
  constexpr int ROWB = F32 ? 128 : 64;           // LDS bytes per operand row per part
  constexpr int A_BYTES = NS * BM * ROWB, B_BYTES = NS * BN * ROWB;   // one buffer
  constexpr int A_UNITS = BM * (kBK / 4);                  // (row, k-quad)
  constexpr int B_UNITS = (kBK / 4) * (BN / 4);            // (k-quad, n-quad)
  constexpr int A_PER = A_UNITS / kThreads;
  constexpr int B_PER = (B_UNITS + kThreads - 1) / kThreads;
  static_assert(A_UNITS % kThreads == 0, "A load split");
  static_assert(B_UNITS % kThreads == 0 || B_UNITS < kThreads, "B load split");
  constexpr int NLD = A_PER + 4 * B_PER;         // 128-bit loads per thread and step
  constexpr int NB = FM * FN;                    // 32x32 blocks per wave
  __shared__ __align__(16) char lds[2 * (A_BYTES + B_BYTES)];

  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wr = (wave / WN) * WTM, wc = (wave % WN) * WTN;   // wave origin in the tile
  const int l32 = lane & 31, lh = lane >> 5;                   // row/col in block, k-half
  const int q = remap_wg(blockIdx.x, nwg, xcd);
  const int it1 = wg_off[q + 1];
  stamp_start(pr, q);

  for (int it = wg_off[q]; it < it1; ++it) {
    const WorkItem W = uni(items[it]);
    const Problem P = uni(get_prob(pr, W.prob));
    const float* A = (const float*)P.A;
    const float* B = (const float*)P.B;
    for (int i0 = W.n0; i0 < W.n1; i0 += BM) {
      for (int j0 = W.m0; j0 < W.m1; j0 += BN) {
        f32x16 acc[FM][FN];
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
          for (int b = 0; b < FN; ++b)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[a][b][e] = 0.f;

        const auto a_rsrc = make_rsrc(A + (int64_t)i0 * P.lda, P.n - i0, P.lda, P.k);
        // A unit u = t + s*kThreads: row u / 8, k-quad t % 8
        const int a_row = t >> 3, a_kq = t & 7;
        const int a_voff0 = (a_row * (int)P.lda + 4 * a_kq) * 4;
        const int a_soff = (kThreads / 8) * (int)P.lda * 4;
        // B unit u = t + s*kThreads: k-quad u % 8, n-quad u / 8
        f32x4 ra[A_PER], rb[B_PER][4];
        int klim = 0, lkk = 0;
        // A step at or past the end of the k-range reads through empty
        // buffer resources (every lane gets 0, no memory is touched), so the
        // pipeline below can fetch one step ahead without a branch.
        const auto a_none = make_rsrc(A, 0, 0, 0);
        __amdgpu_buffer_rsrc_t la = a_none, lb = a_none;
        // prep(kk) sets up the fetch of step kk; load_unit(i) issues its
        // i-th 128-bit load per thread (A units first, then the four rows of
        // each B unit)
        auto prep = [&](int kk) {
          klim = W.k1 - kk;
          lkk = kk;
          const bool live = kk < W.k1;
          la = live ? a_rsrc : a_none;
          lb = make_rsrc(B + (int64_t)kk * P.ldb, live ? P.k - kk : 0, P.ldb, P.m);
        };
        auto load_unit = [&](int i) {
          if (i < A_PER) {
            ra[i] = load4<VEC>(la, a_voff0 + lkk * 4, i * a_soff);
          } else {
            const int s = (i - A_PER) / 4, r = (i - A_PER) % 4;
            const int u = t + s * kThreads;
            if (B_UNITS % kThreads == 0 || u < B_UNITS) {
              const int kq = u & 7, nq = u >> 3;
              const int voff = ((4 * kq) * (int)P.ldb + j0 + 4 * nq) * 4;
              rb[s][r] = load4<VEC>(lb, voff, r * (int)P.ldb * 4);
            }
          }
        };
        // k beyond the piece is zeroed in the registers before the step is
        // stored (a uniform branch, taken on a piece's last step only); rows
        // and columns beyond it are discarded by the epilogue.
        auto mask_regs = [&] {
#pragma unroll
          for (int i = 0; i < A_PER; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
              if (4 * a_kq + j >= klim) ra[i][j] = 0.f;
#pragma unroll
          for (int s = 0; s < B_PER; ++s)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (4 * ((t + s * kThreads) & 7) + r >= klim) rb[s][r] = (f32x4){0.f, 0.f, 0.f, 0.f};
        };
        // store_unit(bsel, i): split and write the data of load unit i (for
        // B: column i % 4 of unit (i - A_PER) / 4, which needs all four of
        // its row loads) into LDS buffer bsel.
        auto store_unit = [&](int bsel, int i) {
          char* As = lds + bsel * (A_BYTES + B_BYTES);
          char* Bs = As + A_BYTES;
          if (i < A_PER) {
            const int row = a_row + i * (kThreads / 8);
            f32x4 v = ra[i];
            if constexpr (F32) {
              *(f32x4*)(As + lds_off<true>(row, a_kq)) = v;
            } else {
              u32x2 parts[NS];
              split4<NS>(v[0], v[1], v[2], v[3], parts);
#pragma unroll
              for (int p = 0; p < NS; ++p)
                *(u32x2*)(As + p * BM * ROWB + lds_off<false>(row, a_kq >> 1) + (a_kq & 1) * 8) = parts[p];
            }
          } else {
            const int s = (i - A_PER) / 4, c = (i - A_PER) % 4;
            const int u = t + s * kThreads;
            if (B_UNITS % kThreads == 0 || u < B_UNITS) {
              const int kq = u & 7, nq = u >> 3;
              float v[4];
#pragma unroll
              for (int r = 0; r < 4; ++r) v[r] = rb[s][r][c];
              const int n = 4 * nq + c;
              if constexpr (F32) {
                *(f32x4*)(Bs + lds_off<true, true>(n, kq)) = (f32x4){v[0], v[1], v[2], v[3]};
              } else {
                u32x2 parts[NS];
                split4<NS>(v[0], v[1], v[2], v[3], parts);
#pragma unroll
                for (int p = 0; p < NS; ++p)
                  *(u32x2*)(Bs + p * BN * ROWB + lds_off<false, true>(n, kq >> 1) + (kq & 1) * 8) = parts[p];
              }
            }
          }
        };
        auto fence = [] { __builtin_amdgcn_sched_barrier(0); };

        // Software pipeline with one barrier per step: while step s is
        // multiplied out of LDS buffer s % 2, step s + 1 (in registers) is
        // split into buffer (s + 1) % 2 and step s + 2 is fetched.
        prep(W.k0);
#pragma unroll
        for (int i = 0; i < NLD; ++i) load_unit(i);
        if (klim < kBK) mask_regs();
#pragma unroll
        for (int i = 0; i < NLD; ++i) store_unit(0, i);
        prep(W.k0 + kBK);
#pragma unroll
        for (int i = 0; i < NLD; ++i) load_unit(i);
        __syncthreads();
        int bsel = 0;
        for (int kk = W.k0; kk < W.k1; kk += kBK) {
          if (klim < kBK) mask_regs();
          const char* As = lds + bsel * (A_BYTES + B_BYTES);
          const char* Bs = As + A_BYTES;
          if constexpr (F32) {
            // lane half lh reads float chunk 2*s + lh (4 k values) of its row;
            // instruction j of the chunk pairs component j of A and B
#pragma unroll
            for (int s = 0; s < 4; ++s) {
              f32x4 fa[FM], fb[FN];
#pragma unroll
              for (int a = 0; a < FM; ++a) fa[a] = *(const f32x4*)(As + lds_off<true>(wr + a * 32 + l32, 2 * s + lh));
#pragma unroll
              for (int b = 0; b < FN; ++b) fb[b] = *(const f32x4*)(Bs + lds_off<true, true>(wc + b * 32 + l32, 2 * s + lh));
              if (s == 0) {
#pragma unroll
                for (int i = 0; i < NLD; ++i) store_unit(bsel ^ 1, i);
                prep(kk + 2 * kBK);
#pragma unroll
                for (int i = 0; i < NLD; ++i) load_unit(i);
              }
#pragma unroll
              for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int b = 0; b < FN; ++b)
#pragma unroll
                  for (int j = 0; j < 4; ++j) acc[a][b] = mfma_f32(fa[a][j], fb[b][j], acc[a][b]);
            }
          } else {
            // Two k-halves of 16; lane half lh reads 16-byte chunk 2*kh + lh.
            // The order is fixed by hand (sched_barrier fences): the first
            // half's blocks each followed by a share of the next step's
            // split-and-store, the second half's A fragments read as soon as
            // the first half's die, then the second half's blocks each
            // followed by a share of the fetch of the step after next.
            auto frag_a = [&](int kh, int a, bf16x8(&f)[NS]) {
#pragma unroll
              for (int p = 0; p < NS; ++p)
                f[p] = *(const bf16x8*)(As + p * BM * ROWB + lds_off<false>(wr + a * 32 + l32, 2 * kh + lh));
            };
            auto frag_b = [&](int kh, int b, bf16x8(&f)[NS]) {
#pragma unroll
              for (int p = 0; p < NS; ++p)
                f[p] = *(const bf16x8*)(Bs + p * BN * ROWB + lds_off<false, true>(wc + b * 32 + l32, 2 * kh + lh));
            };
            auto mma = [&](int a, int b, const bf16x8(&x)[NS], const bf16x8(&y)[NS]) {
              f32x16 c = acc[a][b];
              if constexpr (NS == 2) {
                c = mfma_bf16(x[1], y[0], c);
                c = mfma_bf16(x[0], y[1], c);
                c = mfma_bf16(x[0], y[0], c);
              } else {
                c = mfma_bf16(x[2], y[0], c);
                c = mfma_bf16(x[0], y[2], c);
                c = mfma_bf16(x[1], y[1], c);
                c = mfma_bf16(x[1], y[0], c);
                c = mfma_bf16(x[0], y[1], c);
                c = mfma_bf16(x[0], y[0], c);
              }
              acc[a][b] = c;
            };
            bf16x8 fa0[FM][NS], fb0[FN][NS], fa1[FM][NS], fb1[FN][NS];
#pragma unroll
            for (int a = 0; a < FM; ++a) frag_a(0, a, fa0[a]);
#pragma unroll
            for (int b = 0; b < FN; ++b) frag_b(0, b, fb0[b]);
            fence();
#pragma unroll
            for (int blk = 0; blk < NB; ++blk) {
              const int a = blk / FN, b = blk % FN;
              mma(a, b, fa0[a], fb0[b]);
#pragma unroll
              for (int i = blk * NLD / NB; i < (blk + 1) * NLD / NB; ++i) store_unit(bsel ^ 1, i);
              if (b == FN - 1) frag_a(1, a, fa1[a]);
              fence();
            }
#pragma unroll
            for (int b = 0; b < FN; ++b) frag_b(1, b, fb1[b]);
            prep(kk + 2 * kBK);
            fence();
#pragma unroll
            for (int blk = 0; blk < NB; ++blk) {
              const int a = blk / FN, b = blk % FN;
              mma(a, b, fa1[a], fb1[b]);
#pragma unroll
              for (int i = blk * NLD / NB; i < (blk + 1) * NLD / NB; ++i) load_unit(i);
              fence();
            }
          }
          __syncthreads();
          bsel ^= 1;
        }

        // epilogue: lane holds column l32 of each 32x32 block, value 4g + r
        // in row 8g + 4*lh + r.  Stores go through a buffer resource that
        // starts at the block's first row (a 64-bit address, so the 32-bit
        // offsets stay below 32 rows of the leading dimension) and ends at
        // the piece's last row, so rows past the piece are dropped by the
        // range check; columns past it are skipped per block.
        float* obase;
        int64_t old;
        if (W.out_off < 0) {
          obase = (float*)P.C + (int64_t)i0 * P.ldc;
          old = P.ldc;
        } else {
          old = W.m1 - W.m0;
          obase = ws + W.out_off + (int64_t)(i0 - W.n0) * old - W.m0;
        }
        const bool accum = W.out_off < 0 && P.accumulate;
        auto epilogue = [&](auto accum_c) {
          constexpr bool ACC = decltype(accum_c)::value;
#pragma unroll
          for (int a = 0; a < FM; ++a) {
            const int r0 = wr + a * 32;
            const auto o_rsrc = make_rsrc(obase + (int64_t)r0 * old, W.n1 - i0 - r0, old, W.m1);
#pragma unroll
            for (int b = 0; b < FN; ++b) {
              const int c = j0 + wc + b * 32 + l32;
              if (c >= W.m1) continue;
              const int voff = ((4 * lh) * (int)old + c) * 4;
#pragma unroll
              for (int e = 0; e < 16; ++e) {
                const int soff = (8 * (e >> 2) + (e & 3)) * (int)old * 4;
                float v = acc[a][b][e];
                if constexpr (ACC)
                  v += __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(o_rsrc, voff, soff, 0));
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), o_rsrc, voff, soff, 0);
              }
            }
          }
        };
        if (accum) epilogue(std::true_type{});
        else epilogue(std::false_type{});
      }
    }
    fold_after_item<RSum, kThreads>(pr, it, ws);
  }
  stamp_end(pr, q);
}

template <int PREC, int BM, int BN, int WM, int WN>
hipError_t launch_shape(bool vec, const ProbRef& pr, const WorkItem* items, const int32_t* wg_off, int nwg,
                        int xcd, void* ws, hipStream_t s) {
  dim3 g(nwg), b(64 * WM * WN);
  if (vec)
    hipLaunchKernelGGL((k_ring<PREC, BM, BN, WM, WN, true>), g, b, 0, s, pr, items, wg_off, nwg, xcd, (float*)ws);
  else
    hipLaunchKernelGGL((k_ring<PREC, BM, BN, WM, WN, false>), g, b, 0, s, pr, items, wg_off, nwg, xcd, (float*)ws);
  return hipGetLastError();
}

template <int PREC>
hipError_t launch_prec(int tile, bool vec, const ProbRef& pr, const WorkItem* items, const int32_t* wg_off,
                       int nwg, int xcd, void* ws, hipStream_t s) {
  switch (tile) {
    case RING_T256x128: return launch_shape<PREC, 256, 128, 4, 2>(vec, pr, items, wg_off, nwg, xcd, ws, s);
    case RING_T128x128: return launch_shape<PREC, 128, 128, 4, 2>(vec, pr, items, wg_off, nwg, xcd, ws, s);
    case RING_T128x64: return launch_shape<PREC, 128, 64, 4, 2>(vec, pr, items, wg_off, nwg, xcd, ws, s);
    case RING_T128x128W4: return launch_shape<PREC, 128, 128, 2, 2>(vec, pr, items, wg_off, nwg, xcd, ws, s);
    case RING_T256x256:
      // three bf16 parts of a 256 x 256 tile do not fit the 160 KiB of LDS
      if constexpr (PREC != PREC_BF16X6)
        return launch_shape<PREC, 256, 256, 2, 4>(vec, pr, items, wg_off, nwg, xcd, ws, s);
      break;
  }
  return hipErrorInvalidValue;
}

}  // namespace

RingTileShape ring_tile_shape(int tile, int prec) {
  (void)prec;
  switch (tile) {
    case RING_T256x128: return {256, 128, kBK};
    case RING_T128x128: return {128, 128, kBK};
    case RING_T128x64: return {128, 64, kBK};
    case RING_T128x128W4: return {128, 128, kBK};
    case RING_T256x256: return {256, 256, kBK};
  }
  return {0, 0, 0};
}

hipError_t launch_ring(int prec, int tile, const ProbRef& pr, const WorkItem* items, const int32_t* wg_off,
                       int nwg, int xcd, void* ws, hipStream_t s) {
  if (nwg <= 0) return hipSuccess;
  // 128-bit loads need 16-byte aligned rows and row lengths that are
  // multiples of 4 (so no vector straddles the end of a matrix); the host
  // checks every problem of the launch and sets vec_ok.
  const bool vec = pr.vec_ok != 0;
  switch (prec) {
    case PREC_FP32: return launch_prec<PREC_FP32>(tile, vec, pr, items, wg_off, nwg, xcd, ws, s);
    case PREC_BF16X3: return launch_prec<PREC_BF16X3>(tile, vec, pr, items, wg_off, nwg, xcd, ws, s);
    case PREC_BF16X6: return launch_prec<PREC_BF16X6>(tile, vec, pr, items, wg_off, nwg, xcd, ws, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace paco

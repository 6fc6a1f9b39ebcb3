// k_ring.hip -- persistent (+,x) ring kernel on gfx950 matrix cores.
//
// One workgroup (4 waves, 2 x 2) stands for one processor of the PACO
// partition and runs its cuboid(s): the C face is swept in BM x BN tiles,
// the cuboid's k-range folded 32 at a time.  Operands arrive as float32.
//  FP32   : tiles staged in LDS as float32, v_mfma_f32_16x16x4_f32.
//  BF16X3 : each element is split while it is written to LDS, hi = bf16(x),
//           lo = bf16(x - hi) (round to nearest even; x - hi is exact), and
//           each 16x16 block takes lo*hi', hi*lo', hi*hi' on
//           v_mfma_f32_16x16x32_bf16 with float32 accumulation.
//  BF16X6 : hi, mid = bf16(x - hi), lo = bf16(x - hi - mid) and the six
//           products lo*hi', hi*lo', mid*mid', mid*hi', hi*mid', hi*hi'.
// The split costs no extra HBM pass: global float32 loads for the next step
// are in flight while the current step runs; the split happens on the way
// into LDS.  B is stored k-contiguous (transposed) so both operands are read
// as 8 consecutive k values per lane (one 128-bit LDS read).  Rows of LDS
// tiles are padded so the 16 rows read by a quarter-wave fall on distinct
// banks.
//
// Within a matrix-core instruction each lane group supplies a k-slice; A and
// B use the same lane-to-k assignment, so every k is paired exactly once.
#include "kcommon.h"
#include "kernels.h"

namespace paco {
namespace {

constexpr int kThreads = 256;
constexpr int kBK = 32;

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ __forceinline__ uint16_t bf16_bits(__bf16 h) { return __builtin_bit_cast(uint16_t, h); }
__device__ __forceinline__ float bf16_to_f32(__bf16 h) {
  return __builtin_bit_cast(float, (uint32_t)bf16_bits(h) << 16);
}

// Split 4 float32 values into NS bf16 parts; part p of value j goes to
// out[p] bits [16j, 16j+16).
template <int NS>
__device__ __forceinline__ void split4(const float v[4], uint64_t out[NS]) {
#pragma unroll
  for (int p = 0; p < NS; ++p) out[p] = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float r = v[j];
#pragma unroll
    for (int p = 0; p < NS; ++p) {
      __bf16 h = (__bf16)r;
      out[p] |= (uint64_t)bf16_bits(h) << (16 * j);
      if (p + 1 < NS) r = r - bf16_to_f32(h);
    }
  }
}

__device__ __forceinline__ f32x4 mfma_bf16(const bf16x8& a, const bf16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma_f32(float a, float b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Loads a float32 value range through a buffer resource: VEC issues one
// 128-bit load (16-byte aligned data), otherwise four 32-bit loads.
template <bool VEC>
__device__ __forceinline__ void load4(const __amdgpu_buffer_rsrc_t& r, int voff, int soff, float v[4]) {
  if constexpr (VEC) {
    f32x4 x = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
    v[0] = x[0]; v[1] = x[1]; v[2] = x[2]; v[3] = x[3];
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      v[j] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff + 4 * j, soff, 0));
  }
}

template <int PREC, int BM, int BN, bool VEC>
__global__ __launch_bounds__(kThreads) void k_ring(ProbRef pr, const WorkItem* __restrict__ items,
                                                    const int32_t* __restrict__ wg_off, int nwg, int xcd,
                                                    float* __restrict__ ws) {
  constexpr int NS = PREC == PREC_FP32 ? 1 : (PREC == PREC_BF16X3 ? 2 : 3);
  constexpr bool F32 = PREC == PREC_FP32;
  constexpr int WTM = BM / 2, WTN = BN / 2;      // wave tile
  constexpr int FM = WTM / 16, FN = WTN / 16;    // 16x16 blocks per wave
  // LDS row lengths (elements): bf16 rows of 32 + 8 pad, float rows 32 + 4.
  constexpr int LH = kBK + 8, LF = kBK + 4;
  constexpr int A_UNITS = BM * (kBK / 4);                    // (row, k-quad)
  constexpr int B_UNITS = (kBK / 4) * (BN / 4);              // (k-quad, n-quad)
  constexpr int A_PER = A_UNITS / kThreads, B_PER = (B_UNITS + kThreads - 1) / kThreads;
  static_assert(A_UNITS % kThreads == 0, "load split");
  static_assert(B_UNITS % kThreads == 0 || B_UNITS < kThreads, "load split");

  // bf16 parts: [part][buf][row][LH]; float: [buf][row][LF]
  constexpr int A_H = F32 ? 0 : NS * 2 * BM * LH, B_H = F32 ? 0 : NS * 2 * BN * LH;
  constexpr int A_F = F32 ? 2 * BM * LF : 0, B_F = F32 ? 2 * BN * LF : 0;
  __shared__ __align__(16) uint16_t sh_h[(A_H + B_H) > 0 ? (A_H + B_H) : 8];
  __shared__ __align__(16) float sh_f[(A_F + B_F) > 0 ? (A_F + B_F) : 4];
  uint16_t* Ah = sh_h;
  uint16_t* Bh = sh_h + A_H;
  float* Af = sh_f;
  float* Bf = sh_f + A_F;

  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wr = (wave >> 1) * WTM, wc = (wave & 1) * WTN;   // wave origin in tile
  const int lr = lane & 15, lg = lane >> 4;                   // row/col in block, k-group
  const int q = remap_wg(blockIdx.x, nwg, xcd);
  const int it1 = wg_off[q + 1];
  int buf = 0;

  for (int it = wg_off[q]; it < it1; ++it) {
    const WorkItem W = uni(items[it]);
    const Problem P = uni(get_prob(pr, W.prob));
    const float* A = (const float*)P.A;
    const float* B = (const float*)P.B;
    for (int i0 = W.n0; i0 < W.n1; i0 += BM) {
      for (int j0 = W.m0; j0 < W.m1; j0 += BN) {
        f32x4 acc[FM][FN];
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
          for (int b = 0; b < FN; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

        const auto a_rsrc = make_rsrc(A + (int64_t)i0 * P.lda, P.n - i0, P.lda, P.k);
        // A unit u = t + s*256: row u / 8, k-quad u % 8 (row step 32 per s)
        const int a_row = t / (kBK / 4), a_kq = t % (kBK / 4);
        int a_voff = (a_row * (int)P.lda + W.k0 + 4 * a_kq) * 4;
        const int a_soff = (kThreads / (kBK / 4)) * (int)P.lda * 4;
        // B unit u = t + s*256: n-quad u % (BN/4), k-quad u / (BN/4)
        float ra[A_PER][4], rb[B_PER][4][4];
        int a_klim = 0, b_klim = 0;
        auto load = [&](int kk) {
          a_klim = W.k1 - kk;
#pragma unroll
          for (int s = 0; s < A_PER; ++s) load4<VEC>(a_rsrc, a_voff, s * a_soff, ra[s]);
          a_voff += kBK * 4;
          const auto b_rsrc = make_rsrc(B + (int64_t)kk * P.ldb, P.k - kk, P.ldb, P.m);
          b_klim = W.k1 - kk;
#pragma unroll
          for (int s = 0; s < B_PER; ++s) {
            const int u = t + s * kThreads;
            if (u >= B_UNITS) break;
            const int nq = u % (BN / 4), kq = u / (BN / 4);
            const int voff = ((4 * kq) * (int)P.ldb + j0 + 4 * nq) * 4;
#pragma unroll
            for (int r = 0; r < 4; ++r) load4<VEC>(b_rsrc, voff, r * (int)P.ldb * 4, rb[s][r]);
          }
        };
        auto store = [&]() {
          // A: zero k beyond the piece; rows beyond the piece are discarded
#pragma unroll
          for (int s = 0; s < A_PER; ++s) {
            const int row = a_row + s * (kThreads / (kBK / 4));
            float v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = (4 * a_kq + j < a_klim) ? ra[s][j] : 0.f;
            if constexpr (F32) {
              *(f32x4*)&Af[(buf * BM + row) * LF + 4 * a_kq] = f32x4{v[0], v[1], v[2], v[3]};
            } else {
              uint64_t parts[NS];
              split4<NS>(v, parts);
#pragma unroll
              for (int p = 0; p < NS; ++p)
                *(uint64_t*)&Ah[((p * 2 + buf) * BM + row) * LH + 4 * a_kq] = parts[p];
            }
          }
#pragma unroll
          for (int s = 0; s < B_PER; ++s) {
            const int u = t + s * kThreads;
            if (u >= B_UNITS) break;
            const int nq = u % (BN / 4), kq = u / (BN / 4);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              float v[4];
#pragma unroll
              for (int r = 0; r < 4; ++r) v[r] = (4 * kq + r < b_klim) ? rb[s][r][c] : 0.f;
              const int n = 4 * nq + c;
              if constexpr (F32) {
                *(f32x4*)&Bf[(buf * BN + n) * LF + 4 * kq] = f32x4{v[0], v[1], v[2], v[3]};
              } else {
                uint64_t parts[NS];
                split4<NS>(v, parts);
#pragma unroll
                for (int p = 0; p < NS; ++p)
                  *(uint64_t*)&Bh[((p * 2 + buf) * BN + n) * LH + 4 * kq] = parts[p];
              }
            }
          }
        };

        if (W.k0 < W.k1) load(W.k0);
        for (int kk = W.k0; kk < W.k1; kk += kBK) {
          store();
          __syncthreads();
          if (kk + kBK < W.k1) load(kk + kBK);
          if constexpr (F32) {
#pragma unroll
            for (int kh = 0; kh < kBK / 16; ++kh) {
              f32x4 fa[FM], fb[FN];
#pragma unroll
              for (int a = 0; a < FM; ++a)
                fa[a] = *(const f32x4*)&Af[(buf * BM + wr + a * 16 + lr) * LF + kh * 16 + 4 * lg];
#pragma unroll
              for (int b = 0; b < FN; ++b)
                fb[b] = *(const f32x4*)&Bf[(buf * BN + wc + b * 16 + lr) * LF + kh * 16 + 4 * lg];
#pragma unroll
              for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int b = 0; b < FN; ++b)
#pragma unroll
                  for (int j = 0; j < 4; ++j) acc[a][b] = mfma_f32(fa[a][j], fb[b][j], acc[a][b]);
            }
          } else {
            bf16x8 fa[FM][NS], fb[FN][NS];
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
              for (int p = 0; p < NS; ++p)
                fa[a][p] = *(const bf16x8*)&Ah[((p * 2 + buf) * BM + wr + a * 16 + lr) * LH + 8 * lg];
#pragma unroll
            for (int b = 0; b < FN; ++b)
#pragma unroll
              for (int p = 0; p < NS; ++p)
                fb[b][p] = *(const bf16x8*)&Bh[((p * 2 + buf) * BN + wc + b * 16 + lr) * LH + 8 * lg];
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
              for (int b = 0; b < FN; ++b) {
                f32x4 c = acc[a][b];
                if constexpr (NS == 2) {
                  c = mfma_bf16(fa[a][1], fb[b][0], c);
                  c = mfma_bf16(fa[a][0], fb[b][1], c);
                  c = mfma_bf16(fa[a][0], fb[b][0], c);
                } else {
                  c = mfma_bf16(fa[a][2], fb[b][0], c);
                  c = mfma_bf16(fa[a][0], fb[b][2], c);
                  c = mfma_bf16(fa[a][1], fb[b][1], c);
                  c = mfma_bf16(fa[a][1], fb[b][0], c);
                  c = mfma_bf16(fa[a][0], fb[b][1], c);
                  c = mfma_bf16(fa[a][0], fb[b][0], c);
                }
                acc[a][b] = c;
              }
          }
          buf ^= 1;
        }

        // epilogue: lane holds column lr, rows 4*lg + r of each 16x16 block
        const int64_t tld = W.m1 - W.m0;
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
          for (int b = 0; b < FN; ++b) {
            const int c = j0 + wc + b * 16 + lr;
            if (c >= W.m1) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = i0 + wr + a * 16 + 4 * lg + r;
              if (row >= W.n1) continue;
              float v = acc[a][b][r];
              if (W.out_off < 0) {
                float* cp = (float*)P.C + (int64_t)row * P.ldc + c;
                if (P.accumulate) v = gload(cp) + v;
                gstore(cp, v);
              } else {
                gstore(ws + W.out_off + (int64_t)(row - W.n0) * tld + (c - W.m0), v);
              }
            }
          }
      }
    }
  }
}

template <int PREC, int BM, int BN>
hipError_t launch_shape(bool vec, const ProbRef& pr, const WorkItem* items, const int32_t* wg_off, int nwg,
                        int xcd, void* ws, hipStream_t s) {
  dim3 g(nwg), b(kThreads);
  if (vec)
    hipLaunchKernelGGL((k_ring<PREC, BM, BN, true>), g, b, 0, s, pr, items, wg_off, nwg, xcd, (float*)ws);
  else
    hipLaunchKernelGGL((k_ring<PREC, BM, BN, false>), g, b, 0, s, pr, items, wg_off, nwg, xcd, (float*)ws);
  return hipGetLastError();
}

template <int PREC>
hipError_t launch_prec(int tile, bool vec, const ProbRef& pr, const WorkItem* items, const int32_t* wg_off,
                       int nwg, int xcd, void* ws, hipStream_t s) {
  switch (tile) {
    case RING_T128x128: return launch_shape<PREC, 128, 128>(vec, pr, items, wg_off, nwg, xcd, ws, s);
    case RING_T64x64: return launch_shape<PREC, 64, 64>(vec, pr, items, wg_off, nwg, xcd, ws, s);
    case RING_T256x128:
      // three bf16 parts of a 256 x 128 tile do not fit the 160 KiB of LDS
      if constexpr (PREC != PREC_BF16X6)
        return launch_shape<PREC, 256, 128>(vec, pr, items, wg_off, nwg, xcd, ws, s);
      break;
  }
  return hipErrorInvalidValue;
}

}  // namespace

RingTileShape ring_tile_shape(int tile, int prec) {
  (void)prec;
  switch (tile) {
    case RING_T128x128: return {128, 128, kBK};
    case RING_T64x64: return {64, 64, kBK};
    case RING_T256x128: return {256, 128, kBK};
  }
  return {0, 0, 0};
}

hipError_t launch_ring(int prec, int tile, const ProbRef& pr, const WorkItem* items, const int32_t* wg_off,
                       int nwg, int xcd, void* ws, hipStream_t s) {
  if (nwg <= 0) return hipSuccess;
  // 128-bit loads need 16-byte aligned rows and row lengths that are
  // multiples of 4 (so no vector straddles the end of a matrix); batched
  // problems use the base problem's layout.
  const Problem& b = pr.base;
  bool vec = pr.table == nullptr && ((uintptr_t)b.A % 16 == 0) && ((uintptr_t)b.B % 16 == 0) &&
             b.lda % 4 == 0 && b.ldb % 4 == 0 && b.k % 4 == 0 && b.m % 4 == 0 && pr.sA % 4 == 0 &&
             pr.sB % 4 == 0;
  switch (prec) {
    case PREC_FP32: return launch_prec<PREC_FP32>(tile, vec, pr, items, wg_off, nwg, xcd, ws, s);
    case PREC_BF16X3: return launch_prec<PREC_BF16X3>(tile, vec, pr, items, wg_off, nwg, xcd, ws, s);
    case PREC_BF16X6: return launch_prec<PREC_BF16X6>(tile, vec, pr, items, wg_off, nwg, xcd, ws, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace paco

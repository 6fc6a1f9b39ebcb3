// k_dp1d.hip -- the 1D problem (section "PACO 1D", equation (1D)):
// D[j] = min over i < j of D[i] + w(i, j), with w computed in registers.
//
// The recursion of the section, in order, alternates base triangles (a short
// run of outputs finished inside one workgroup) and squares (the finished
// inputs of a left half applied to the outputs of its right half).  One
// launch covers one square, one workgroup per PACO piece, and the base
// triangle that follows it: the last workgroup to finish its piece (an
// atomic count, reset by that workgroup) runs the triangle.  No workgroup
// ever waits for another, so the launch drains whatever the residency.
//
// Values are unsigned 32-bit with INF = 2^30 as "no path": w <= 2^30 (the
// host checks), so every sum stays below 2^31, and stored values are
// clamped to INF.  Square outputs combine with device-scope atomic minima
// (exact: min is associative, commutative and idempotent), which also makes
// them visible to the triangle that reads them with device-scope loads.
#include "kcommon.h"
#include "kernels.h"

namespace paco {
namespace {

constexpr uint32_t DP_INF = 1u << 30;
constexpr uint32_t DP_KEY_MUL = 0x9E3779B9u;

// MurmurHash3's 32-bit finaliser (Appleby)
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h;
}

// w(i, j); WK 0: a + b (j - i); WK 1: a + (fmix32((i K + j) ^ seed) & mask)
template <int WK>
__device__ __forceinline__ uint32_t wval(const DpW& w, uint32_t i, uint32_t j) {
  if constexpr (WK == 0) {
    return w.a + w.b * (j - i);
  } else {
    return w.a + (fmix32((i * DP_KEY_MUL + j) ^ w.seed) & w.b);
  }
}

__device__ __forceinline__ uint32_t umin(uint32_t x, uint32_t y) { return x < y ? x : y; }

__device__ __forceinline__ uint32_t load_dev(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Inputs [i0 + t0, i0 + t0 + cnt) of a finished block (lane t of `vin`
// holds input i0 + t; affine: with -b i folded in) applied to the outputs
// [o_beg, len) of the triangle, merged into d by LDS atomic minima.  cnt <=
// MAXK; slots past cnt take 2^31, which no sum with a weight <= 2^30 brings
// below a real candidate.
template <int WK, int MAXK>
__device__ __forceinline__ void tri_apply(uint32_t vin, int t0, int cnt, uint32_t i0, int64_t lo, int o_beg, int len,
                                          const DpW& w, uint32_t* d) {
  const int lane = threadIdx.x & 63;
  uint32_t sv[MAXK];
#pragma unroll
  for (int k = 0; k < MAXK; ++k)
    sv[k] = k < cnt ? (uint32_t)__builtin_amdgcn_readlane((int)vin, t0 + k) : 0x80000000u;
#pragma unroll 1
  for (int o0 = o_beg; o0 < len; o0 += 64) {
    const int o = o0 + lane;
    const uint32_t j = (uint32_t)(lo + o);
    uint32_t acc = DP_INF;
    if constexpr (WK == 0) {
      const uint32_t cj = w.a + w.b * j;
#pragma unroll
      for (int k = 0; k < MAXK; ++k) acc = umin(acc, sv[k] + cj);
    } else {
#pragma unroll
      for (int k = 0; k < MAXK; ++k) acc = umin(acc, sv[k] + wval<WK>(w, i0 + (uint32_t)(t0 + k), j));
    }
    if (o < len) atomicMin(d + o, acc);
  }
}

// A base triangle: positions [lo, lo + len), len <= DP_TRI_MAX, whose values
// already hold every update from inputs below lo; run by all 256 threads of
// one workgroup.  Per block of 64 outputs:
//  1. all waves write the block's own weights w(blk + t, blk + l), t < l, to
//     LDS (2^31 where t >= l: dt + 2^31 < 2^32 never wins a minimum);
//  2. wave 0 walks the chain: output t is final once every earlier output of
//     the block has been applied to it, so lane t's value is read as a
//     wave-uniform scalar and applied to the lanes after it.  Meanwhile waves
//     1-3 apply the previous block (22, 21 and 21 of its inputs) to every
//     output after this block;
//  3. all four waves apply this block (16 inputs each) to the next block's
//     64 outputs only, so that the next chain can start.
// An input block thus reaches the next block at step 3 and every later one
// during the next block's chain; the waves' minima meet by LDS atomic minima.
template <int WK>
__device__ void tri_body(uint32_t* __restrict__ D, int64_t lo, int len, const DpW& w, uint32_t* d,
                         uint32_t* wl) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (int t = tid; t < len; t += 256) d[t] = umin(load_dev(D + lo + t), DP_INF);
  for (int blk = 0; blk < len; blk += 64) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = tid + 256 * q;
      const int t = e >> 6, l = e & 63;
      wl[e] = l > t ? wval<WK>(w, (uint32_t)(lo + blk + t), (uint32_t)(lo + blk + l)) : 0x80000000u;
    }
    __syncthreads();   // weights written; d holds every update of earlier blocks
    if (wv == 0) {
      uint32_t acc = blk + lane < len ? d[blk + lane] : DP_INF;
      // weights in chunks of 16 steps, the next chunk requested before the
      // current one is walked (32 registers instead of 64)
      uint32_t wa[16], wb[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) wa[t] = wl[t * 64 + lane];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (c < 3) {
#pragma unroll
          for (int t = 0; t < 16; ++t) wb[t] = wl[(16 * (c + 1) + t) * 64 + lane];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          const uint32_t dt = (uint32_t)__builtin_amdgcn_readlane((int)acc, 16 * c + t);
          acc = umin(acc, dt + wa[t]);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int t = 0; t < 16; ++t) wa[t] = wb[t];
      }
      if (blk + lane < len) d[blk + lane] = umin(acc, DP_INF);
    } else if (blk >= 64 && blk + 64 < len) {
      // the previous block's inputs reach every output after this block
      const int pb = blk - 64;
      const uint32_t i0 = (uint32_t)(lo + pb);
      const uint32_t vin = WK == 0 ? d[pb + lane] - w.b * (i0 + (uint32_t)lane) : d[pb + lane];
      const int t0 = wv == 1 ? 0 : (wv == 2 ? 22 : 43);
      tri_apply<WK, 22>(vin, t0, wv == 1 ? 22 : 21, i0, lo, blk + 64, len, w, d);
    }
    __syncthreads();   // the block is final; the previous block reached every later output
    if (blk + 64 < len) {
      const uint32_t i0 = (uint32_t)(lo + blk);
      // lane t: input blk + t; affine weights fold their input-only part
      // -b i into it, so D[i] + w(i, j) = vin_t + (a + b j)
      const uint32_t vin = WK == 0 ? d[blk + lane] - w.b * (i0 + (uint32_t)lane) : d[blk + lane];
      const int nxt = blk + 128 < len ? blk + 128 : len;
      tri_apply<WK, 16>(vin, 16 * wv, 16, i0, lo, blk + 64, nxt, w, d);
    }
    // the next block's weight pass touches only wl, which nothing reads now;
    // its barrier orders these minima before the next chain
  }
  __syncthreads();
  for (int t = tid; t < len; t += 256) D[lo + t] = d[t];
}

// After this workgroup's updates: count it, and if it is the last of the
// `total` workgroups counted, reset the count and run the triangle.
template <int WK>
__device__ void last_runs_tri(uint32_t* __restrict__ D, uint32_t* __restrict__ cnt, uint32_t total,
                              int64_t tri_lo, int tri_len, const DpW& w, uint32_t* d, uint32_t* wl) {
  __shared__ int s_last;
  __syncthreads();   // every update of this workgroup is complete
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t old = atomicAdd(cnt, 1u);
    s_last = old == total - 1;
    if (s_last) {
      atomicExch(cnt, 0u);
      __threadfence();
    }
  }
  __syncthreads();
  if (s_last && tri_len > 0) tri_body<WK>(D, tri_lo, tri_len, w, d, wl);
}

// D[1..n] = INF, then the first base triangle
template <int WK>
__global__ __launch_bounds__(256) void k_dp1d_fill(uint32_t* __restrict__ D, int64_t n, uint32_t* __restrict__ cnt,
                                                   int tri_len, DpW w) {
  __shared__ uint32_t d[DP_TRI_MAX];
  __shared__ uint32_t wl[64 * 64];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = 1 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j <= n; j += stride)
    __hip_atomic_store(D + j, DP_INF, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  last_runs_tri<WK>(D, cnt, gridDim.x, 0, tri_len, w, d, wl);
}

// External update of one square by its PACO pieces (one per workgroup):
// outputs [j0, j1) take the minimum over the finished inputs [i0, i1).  A
// wave takes a group of DP_R strips of 64 outputs (DP_R per lane) and a
// slice of the inputs, which it reads as wave-uniform values 16 at a time:
// the scalar work per input (its value, the input-only part of w) is shared
// by the DP_R outputs of each lane.  Fewer than four groups split their
// inputs over the waves.  The first `ntri` pieces are those whose outputs
// reach into the base triangle that follows: the last of them to finish
// runs it while the other pieces go on.
constexpr int DP_R = 4;

// one input i applied to a lane's DP_R outputs
template <int WK>
__device__ __forceinline__ void rect_in(uint32_t (&acc)[DP_R], uint32_t di, uint32_t iu, const uint32_t (&ju)[DP_R],
                                        const uint32_t (&cj)[DP_R], const DpW& w) {
  if constexpr (WK == 0) {
    // D[i] + a + b (j - i) = (D[i] - b i) + (a + b j), exact modulo 2^32
    const uint32_t si = di - w.b * iu;
#pragma unroll
    for (int r = 0; r < DP_R; ++r) acc[r] = umin(acc[r], si + cj[r]);
  } else {
    const uint32_t da = di + w.a;
    const uint32_t ki = iu * DP_KEY_MUL;
#pragma unroll
    for (int r = 0; r < DP_R; ++r) acc[r] = umin(acc[r], da + (fmix32((ki + ju[r]) ^ w.seed) & w.b));
  }
}

template <int WK>
__global__ __launch_bounds__(256) void k_dp1d_rect(const uint32_t* __restrict__ Din, uint32_t* __restrict__ Dout,
                                                   const DpPiece* __restrict__ pieces, int ntri,
                                                   uint32_t* __restrict__ cnt, int64_t tri_lo, int tri_len, DpW w) {
  __shared__ uint32_t d[DP_TRI_MAX];
  __shared__ uint32_t wl[64 * 64];
  const DpPiece pc = pieces[blockIdx.x];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t W = pc.j1 - pc.j0, H = pc.i1 - pc.i0;
  if (W > 0 && H > 0) {
    const int64_t groups = (W + 64 * DP_R - 1) / (64 * DP_R);
    const int S = groups >= 4 ? 1 : (groups >= 2 ? 2 : 4);
    const int64_t units = groups * S;
    for (int64_t u = wv; u < units; u += 4) {
      const int64_t g = u / S;
      const int slice = (int)(u - g * S);
      const int64_t jb = pc.j0 + g * 64 * DP_R + lane;
      const int64_t ia = pc.i0 + H * slice / S, ib = pc.i0 + H * (slice + 1) / S;
      uint32_t ju[DP_R], cj[DP_R], acc[DP_R];
#pragma unroll
      for (int r = 0; r < DP_R; ++r) {
        ju[r] = (uint32_t)(jb + 64 * r);
        cj[r] = WK == 0 ? w.a + w.b * ju[r] : 0u;   // affine: the output-only part
        acc[r] = DP_INF;
      }
      // inputs in chunks of CH (one wave-uniform load each), then the rest;
      // affine: two sets of CH alternate, each requested while the other is
      // applied (a pair is about two instructions, too few to cover a load)
      constexpr int CH = WK == 0 ? 16 : 8;
      int64_t i = ia;
      if constexpr (WK == 0) {
        if (i + 2 * CH <= ib) {
          uint32_t va[CH], vb[CH];
#pragma unroll
          for (int k = 0; k < CH; ++k) va[k] = Din[i + k];
          for (; i + 2 * CH <= ib; i += 2 * CH) {
#pragma unroll
            for (int k = 0; k < CH; ++k) vb[k] = Din[i + CH + k];
#pragma unroll
            for (int k = 0; k < CH; ++k) rect_in<WK>(acc, va[k], (uint32_t)(i + k), ju, cj, w);
            if (i + 4 * CH <= ib) {
#pragma unroll
              for (int k = 0; k < CH; ++k) va[k] = Din[i + 2 * CH + k];
            }
#pragma unroll
            for (int k = 0; k < CH; ++k) rect_in<WK>(acc, vb[k], (uint32_t)(i + CH + k), ju, cj, w);
          }
        }
      }
      for (; i + CH <= ib; i += CH) {
        uint32_t dv[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) dv[k] = Din[i + k];
#pragma unroll
        for (int k = 0; k < CH; ++k) rect_in<WK>(acc, dv[k], (uint32_t)(i + k), ju, cj, w);
      }
      for (; i < ib; ++i) rect_in<WK>(acc, Din[i], (uint32_t)i, ju, cj, w);
#pragma unroll
      for (int r = 0; r < DP_R; ++r)
        if (jb + 64 * r < pc.j1) atomicMin(Dout + jb + 64 * r, umin(acc[r], DP_INF));
    }
  }
  if ((int)blockIdx.x < ntri) last_runs_tri<WK>(Dout, cnt, (uint32_t)ntri, tri_lo, tri_len, w, d, wl);
}

}  // namespace

hipError_t launch_dp1d_fill(int wk, uint32_t* D, int64_t n, uint32_t* cnt, int tri_len, const DpW& w,
                            hipStream_t s) {
  if (n < 0 || tri_len < 0 || tri_len > DP_TRI_MAX) return hipErrorInvalidValue;
  const int64_t blocks = (n + 255) / 256;
  const unsigned g = (unsigned)(blocks < 1 ? 1 : (blocks < 1024 ? blocks : 1024));
  if (wk == 0) {
    hipLaunchKernelGGL(k_dp1d_fill<0>, dim3(g), dim3(256), 0, s, D, n, cnt, tri_len, w);
  } else {
    hipLaunchKernelGGL(k_dp1d_fill<1>, dim3(g), dim3(256), 0, s, D, n, cnt, tri_len, w);
  }
  return hipGetLastError();
}

hipError_t launch_dp1d_rect(int wk, uint32_t* D, const DpPiece* pieces, int npieces, int ntri, uint32_t* cnt,
                            int64_t tri_lo, int tri_len, const DpW& w, hipStream_t s) {
  if (npieces <= 0 || ntri < 1 || ntri > npieces || tri_len < 0 || tri_len > DP_TRI_MAX)
    return hipErrorInvalidValue;
  if (wk == 0) {
    hipLaunchKernelGGL(k_dp1d_rect<0>, dim3(npieces), dim3(256), 0, s, D, D, pieces, ntri, cnt, tri_lo, tri_len, w);
  } else {
    hipLaunchKernelGGL(k_dp1d_rect<1>, dim3(npieces), dim3(256), 0, s, D, D, pieces, ntri, cnt, tri_lo, tri_len, w);
  }
  return hipGetLastError();
}

}  // namespace paco

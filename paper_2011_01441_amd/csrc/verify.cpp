// verify.cpp -- sampled-row float64 error report for ring results, and the
// tile choosers of the boolean and ring kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/paco.h"
#include "ctx.h"
#include "kernels.h"

using namespace paco;

namespace paco {

namespace {

paco_status run_verify(paco_ctx ctx, int64_t n, int64_t m, int64_t k, const float* A, int64_t lda,
                       const float* B, int64_t ldb, const float* C, int64_t ldc, const int64_t* d_rows,
                       int64_t nrows, double out[4]) {
  const int64_t nb = verify_blocks(m, nrows);
  hipError_t e;
  if (nb > ctx->rows_cap / 4 || !ctx->d_verify) {
    if (ctx->d_verify) (void)hipFree(ctx->d_verify);
    ctx->d_verify = nullptr;
    if ((e = hipMalloc((void**)&ctx->d_verify, sizeof(double) * 4 * nb)) != hipSuccess)
      return hip_fail(ctx, e, "verify alloc");
    ctx->rows_cap = 4 * nb;
  }
  if ((e = launch_verify_f64(n, m, k, A, lda, B, ldb, C, ldc, d_rows, nrows, ctx->d_verify, ctx->stream)) !=
      hipSuccess)
    return hip_fail(ctx, e, "verify launch");
  std::vector<double> part(4 * nb);
  if ((e = hipMemcpyAsync(part.data(), ctx->d_verify, sizeof(double) * 4 * nb, hipMemcpyDeviceToHost,
                          ctx->stream)) != hipSuccess)
    return hip_fail(ctx, e, "verify copy");
  if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return hip_fail(ctx, e, "verify sync");
  out[0] = out[1] = out[2] = out[3] = 0.0;
  for (int64_t b = 0; b < nb; ++b) {
    out[0] = std::max(out[0], part[4 * b]);
    out[1] = std::max(out[1], part[4 * b + 1]);
    out[2] += part[4 * b + 2];
    out[3] += part[4 * b + 3];
  }
  return PACO_OK;
}

}  // namespace

paco_status verify_sampled(paco_ctx ctx, int64_t n, int64_t m, int64_t k, const float* A, int64_t lda,
                           const float* B, int64_t ldb, const float* C, int64_t ldc, int rows, uint64_t seed,
                           paco_mm_result* res) {
  // distinct rows drawn with splitmix64 from the seed (all rows if fewer)
  std::vector<int64_t> pick;
  if (rows >= n) {
    for (int64_t i = 0; i < n; ++i) pick.push_back(i);
  } else {
    std::vector<char> used(n, 0);
    uint64_t x = seed;
    while ((int64_t)pick.size() < rows) {
      x += 0x9E3779B97F4A7C15ull;
      uint64_t z = x;
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
      z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
      z ^= z >> 31;
      int64_t i = (int64_t)(z % (uint64_t)n);
      if (!used[i]) {
        used[i] = 1;
        pick.push_back(i);
      }
    }
  }
  hipError_t e;
  int64_t* d_rows = nullptr;
  if ((e = hipMalloc((void**)&d_rows, sizeof(int64_t) * pick.size())) != hipSuccess)
    return hip_fail(ctx, e, "verify rows alloc");
  e = hipMemcpy(d_rows, pick.data(), sizeof(int64_t) * pick.size(), hipMemcpyHostToDevice);
  double out[4];
  paco_status st = PACO_OK;
  if (e != hipSuccess) st = hip_fail(ctx, e, "verify rows copy");
  else st = run_verify(ctx, n, m, k, A, lda, B, ldb, C, ldc, d_rows, (int64_t)pick.size(), out);
  (void)hipFree(d_rows);
  if (st != PACO_OK) return st;
  if (res) {
    res->verify_max_rel = out[0];
    res->verify_max_abs = out[1];
  }
  return PACO_OK;
}

namespace {
template <class Shape>
int choose_tile(const std::vector<Piece>& pcs, const int* cand, const double* eff, int nc, Shape shape) {
  int best = cand[0];
  double bestc = 1e300;
  for (int c = 0; c < nc; ++c) {
    int tm, tn;
    shape(cand[c], tm, tn);
    // padded work of the busiest processor (a processor may hold several
    // pieces in multi-piece mode)
    int np = 0;
    for (const Piece& p : pcs) np = std::max(np, p.proc + 1);
    std::vector<double> load(np, 0.0);
    double worst = 0;
    for (const Piece& p : pcs) {
      if (p.empty()) continue;
      double tiles = (double)((p.n1 - p.n0 + tm - 1) / tm) * (double)((p.m1 - p.m0 + tn - 1) / tn);
      load[p.proc] += tiles * tm * tn * (double)(p.k1 - p.k0) * eff[c];
      worst = std::max(worst, load[p.proc]);
    }
    if (worst < bestc) {
      bestc = worst;
      best = cand[c];
    }
  }
  return best;
}
}  // namespace

int choose_bool_tile(const std::vector<Piece>& pcs) {
  const int cand[4] = {BOOL_T512x32W, BOOL_T128x128W, BOOL_T256x64W, BOOL_T64x64W};
  const double eff[4] = {1.0, 1.0, 1.0, 1.4};
  return choose_tile(pcs, cand, eff, 4, [](int t, int& tm, int& tn) {
    BoolTileShape s = bool_tile_shape(t);
    tm = s.tm;
    tn = s.tnw;
  });
}

int choose_ring_tile(const std::vector<Piece>& pcs, int prec) {
  const int cand[4] = {RING_T256x256, RING_T256x128, RING_T128x128, RING_T128x64};
  const double eff[4] = {1.0, 1.1, 1.25, 1.6};
  const int nc = prec == PREC_BF16X6 ? 3 : 4;   // no 256 x 256 for three parts
  return choose_tile(pcs, cand + (4 - nc), eff + (4 - nc), nc, [prec](int t, int& tm, int& tn) {
    RingTileShape s = ring_tile_shape(t, prec);
    tm = s.tm;
    tn = s.tn;
  });
}

}  // namespace paco

extern "C" paco_status paco_verify_rows_f64(paco_ctx ctx, int64_t n, int64_t m, int64_t k, const float* A,
                                            const float* B, const float* C, const int64_t* rows, int64_t nrows,
                                            double* out) {
  if (!ctx) return PACO_ERR_INVALID_ARG;
  if (n < 0 || m < 0 || k < 0 || nrows < 0 || !out || (nrows > 0 && (!rows || !A || !B || !C))) {
    set_err(ctx, "invalid verify arguments");
    return PACO_ERR_INVALID_ARG;
  }
  out[0] = out[1] = out[2] = out[3] = 0.0;
  if (nrows == 0 || m == 0) return PACO_OK;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  // the row list is checked on the host before any kernel reads through it
  std::vector<int64_t> h(nrows);
  if ((e = hipMemcpy(h.data(), rows, sizeof(int64_t) * nrows, hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(ctx, e, "verify rows copy");
  for (int64_t r : h)
    if (r < 0 || r >= n) {
      set_err(ctx, "verify row index out of range");
      return PACO_ERR_INVALID_ARG;
    }
  return run_verify(ctx, n, m, k, A, k, B, m, C, m, rows, nrows, out);
}

// ctx.h -- internal state of a libpaco context.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/paco.h"
#include "partition.h"
#include "plan.h"

namespace paco {

// A cached plan: host work lists and their device copies.
struct DevPlan {
  HostPlan h;
  int tile = 0;
  int fam = 0;  // 0 integer VALU, 1 boolean, 2 ring
  int p = 0;
  double kcut = 0.0;   // k-cut cost the partition used (PACO mode)
  WorkItem* d_items = nullptr;
  int32_t* d_wg_off = nullptr;
  RedTile* d_tiles = nullptr;
  RedSrc* d_srcs = nullptr;
  int32_t* d_item_fold = nullptr;   // fused folding (HostPlan::fused)
  int32_t* d_fold_list = nullptr;
  uint32_t* d_fold_cnt = nullptr;
  virtual ~DevPlan();
};

// A plan whose device tables are not allocated: one host block holding the
// tables (copied to fixed scratch memory at each call) and the offsets of
// each table and of the temporary faces in that memory.
struct HostTables {
  DevPlan plan;   // device pointers stay null
  std::vector<unsigned char> blob;
  uint64_t items_off = 0, wg_off = 0, tiles_off = 0, srcs_off = 0, faces_off = 0;
  uint64_t item_fold_off = 0, fold_list_off = 0, fold_cnt_off = 0;
};

// Caller-provided device memory for a call that allocates nothing.
struct FixedScratch {
  void* ptr;
  uint64_t bytes;
};

}  // namespace paco

struct paco_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  hipEvent_t switch_ev = nullptr;   // orders work across a change of stream (paco_set_stream)
  int num_cus = 0;
  double search_min_gain = 2e-5;   // ring plans: see ring_partition (a server's context plans every request anew)
  uint64_t* stamps = nullptr;    // paco_set_piece_stamps: per-processor timestamps of semiring MM calls
  int32_t stamp_cap = 0;
  std::vector<double> weights;   // processor throughputs for default-p ring calls (paco_set_processor_weights)
  struct Tuned {                 // paco_tune's choice for a shape, used by default calls
    int part = 0, p = 0, tile = -1;
    double kcut = 0.0;
    bool weighted = false;
  };
  std::map<std::string, Tuned> tuned;
  uint64_t budget = 0;
  void* ws = nullptr;        // temporary faces
  uint64_t ws_bytes = 0;
  void* sws = nullptr;       // Strassen temporaries
  uint64_t sws_bytes = 0;
  void* gws = nullptr;       // GAP problem: transposed copy of the final values
  uint64_t gws_bytes = 0;
  double* d_verify = nullptr;  // 4 doubles + row list
  int64_t* d_rows = nullptr;
  int64_t rows_cap = 0;
  std::map<std::string, std::unique_ptr<paco::DevPlan>> plans;
  std::map<std::string, std::unique_ptr<paco::HostTables>> host_plans;   // paco_semiring_mm_noalloc
  std::string last_error;
  // per-kernel timing (paco_timing_enable)
  bool timing = false;
  uint64_t ws_gen = 0;   // bumped whenever ws or sws is (re)allocated: captured graphs check it
  struct Mark {
    hipEvent_t a, b;
    int role;  // 0 main, 1 reduce, 2 other
  };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> event_pool;
};

namespace paco {

// plans a context keeps before it synchronises the device and starts over
constexpr size_t PACO_PLAN_CACHE_MAX = 512;
void trim_plans(paco_ctx ctx);
void set_err(paco_ctx ctx, const std::string& msg);
paco_status hip_fail(paco_ctx ctx, hipError_t e, const char* what);
paco_status upload_plan(paco_ctx ctx, DevPlan* dp);
paco_status ensure_ws(paco_ctx ctx, uint64_t bytes);
int choose_int_tile(const std::vector<Piece>& pcs);
int choose_bool_tile(const std::vector<Piece>& pcs);
int choose_ring_tile(const std::vector<Piece>& pcs, int prec);
// MM-1-Piece of a ring product on the matrix-core kernel's tile grid (the
// tile chosen, or the forced one); the dimension search runs when it may
// save more than min_gain_s of kernel time (plans of library calls are
// cached per shape; the server plans every request anew).
std::vector<Piece> ring_partition(int64_t n, int64_t m, int64_t k, int p, int prec, double kcut_cost,
                                  const double* weights, int force_tile, int* tile_out, double min_gain_s = 2e-5);
paco_status verify_sampled(paco_ctx ctx, int64_t n, int64_t m, int64_t k, const float* A, int64_t lda,
                           const float* B, int64_t ldb, const float* C, int64_t ldc, int rows,
                           uint64_t seed, paco_mm_result* res);
void destroy_ctx_extras(paco_ctx ctx);
int64_t words(int64_t bits);
int auto_precision(int64_t k);
bool ring_vec_ok(const void* A, int64_t lda, const void* B, int64_t ldb, int64_t m, int64_t k);
void make_mm_plan(int sr, int64_t n, int64_t m, int64_t k, int part, int p, int split_k, int prec,
                  int num_cus, DevPlan* np, double kcut_cost, const double* weights = nullptr,
                  int force_tile = -1, double search_min_gain_s = 2e-5);
double default_kcut_cost(int sr);
double plan_kcut_cost(int sr);
// The semiring MM call; force_tile >= 0 fixes the kernel tile (tuning).
// With fx, the plan's tables and temporary faces go to that memory and the
// call allocates no device memory (PACO_ERR_BUDGET when they do not fit).
paco_status run_mm(paco_ctx ctx, const paco_mm_desc* d, paco_mm_result* res, int force_tile = -1,
                   const FixedScratch* fx = nullptr);
void pack_tables(HostTables* t);
// Per-device address of the fixed scratch array (noalloc.cpp); called by
// paco_create with the device current.
paco_status noalloc_init(paco_ctx ctx);
// key of paco_tune's choices
std::string tune_key(const paco_mm_desc* d, int prec);

// Brackets one kernel launch with timing events when timing is enabled.
struct TimeScope {
  paco_ctx ctx;
  int role;
  hipEvent_t a = nullptr;
  TimeScope(paco_ctx c, int r);
  ~TimeScope();
};

}  // namespace paco

// server.cpp -- batching request server (include/paco_server.h).
//
// A dispatcher thread forms batches from the admitted head of the queue and
// launches them; a completion thread waits for each batch's event, stamps
// completion times and returns the batch's bytes to the admission budget.
// At most two batches are in flight, so the next batch is planned and
// uploaded while the previous one runs.  Each batch is split over the
// processors by batch_partition; every semiring group of the batch is one
// persistent launch on its own stream, all groups of a batch concurrent.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/paco.h"
#include "../../include/paco_server.h"
#include "batch.h"
#include "ctx.h"
#include "kernels.h"

using namespace paco;

extern "C" double paco_server_clock(void) {
  using namespace std::chrono;
  static const steady_clock::time_point t0 = steady_clock::now();
  return duration<double>(steady_clock::now() - t0).count();
}

namespace {

constexpr int kSlots = 3;          // descriptor buffers (at most 2 batches in flight)
constexpr size_t kKeepFinished = 1 << 16;   // finished, unpolled requests kept

// Latency histogram: 256 bins per octave from 0.1 us (quantiles within
// 0.3% of the exact order statistic), fixed memory whatever the count.
struct LatHist {
  static constexpr int kPerOct = 256;
  static constexpr int kBins = 42 * kPerOct;   // 0.1 us .. 4.4e5 s
  static constexpr double kMin = 1e-7;
  std::vector<uint32_t> bins = std::vector<uint32_t>(kBins, 0);
  uint64_t count = 0;
  double maxv = 0.0;
  void add(double v) {
    int b = 0;
    if (v > kMin) b = std::min(kBins - 1, 1 + (int)(std::log2(v / kMin) * kPerOct));
    bins[b] += 1;
    count += 1;
    maxv = std::max(maxv, v);
  }
  // the order statistic of rank round(f (count - 1)), as the geometric
  // centre of its bin (bin 0 reads as kMin)
  double quantile(double f) const {
    if (count == 0) return 0.0;
    const uint64_t rank = std::min<uint64_t>(count - 1, (uint64_t)(f * (double)(count - 1) + 0.5));
    uint64_t cum = 0;
    for (int b = 0; b < kBins; ++b) {
      cum += bins[b];
      if (cum > rank) return b == 0 ? kMin : std::min(maxv, kMin * std::exp2((b - 0.5) / kPerOct));
    }
    return maxv;
  }
};

struct ReqState {
  paco_request r;
  int64_t mu, ku;                  // kernel-unit widths (bool: words)
  uint64_t bytes = 0;
  paco_request_result res;
  bool finished = false;
};

// Descriptor blobs up to this size are read by the kernels straight from
// coherent pinned host memory (a handful of reads per workgroup), saving
// the copy to device memory and its host call.
constexpr size_t kZeroCopyBytes = 64 << 10;

struct Slot {
  void* dev = nullptr;             // device descriptor buffer
  void* host = nullptr;            // pinned staging buffer
  size_t cap = 0;
  void* zhost = nullptr;           // coherent pinned buffer of kZeroCopyBytes
  void* zdev = nullptr;            // its device address
  hipEvent_t done = nullptr;       // last batch that used the slot
  bool used = false;
};

struct Batch {
  std::vector<uint64_t> tickets;
  hipEvent_t ev = nullptr;
  bool ok = true;
  int id = 0;
};

uint64_t req_bytes(const paco_request& r, int64_t mu, int64_t ku) {
  const int64_t lda = r.lda ? r.lda : ku, ldb = r.ldb ? r.ldb : mu, ldc = r.ldc ? r.ldc : mu;
  return 4ull * (uint64_t)(r.n * lda + r.k * ldb + r.n * ldc);
}

}  // namespace

struct paco_server_s {
  paco_ctx ctx = nullptr;          // private context (streams, workspace)
  paco_server_opts o{};
  int device = 0, p = 0;
  hipStream_t main = nullptr;
  hipStream_t gs[G_COUNT] = {};
  hipEvent_t ready = nullptr;
  hipEvent_t gdone[G_COUNT] = {};
  Slot slots[kSlots];
  int next_slot = 0;
  void* ws = nullptr;
  uint64_t ws_bytes = 0;

  std::mutex mu;
  std::condition_variable cv;      // queue / budget / in-flight changes
  std::condition_variable cv_done; // completions
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, ReqState> reqs;
  std::deque<Batch> inflight;
  uint64_t next_ticket = 1;
  uint64_t bytes_in_flight = 0;
  int64_t pending = 0;             // submitted, not finished
  bool stop = false;
  bool disp_done = false;          // dispatcher has exited (set under mu)
  int batch_counter = 0;
  // stats
  int64_t submitted = 0, completed = 0, failed = 0, batches = 0, batched_reqs = 0;
  LatHist lat;
  std::deque<uint64_t> finished_order;   // finished tickets, oldest first (retention)
  int32_t fail_next = 0;                 // test hook: batches to fail before launch
  double first_arrival = -1, last_done = 0, ops = 0;

  std::thread dispatcher, completer;
};

namespace {

paco_status grow_slot(paco_server s, Slot& sl, size_t bytes) {
  if (bytes <= sl.cap) return PACO_OK;
  if (sl.used && sl.done) (void)hipEventSynchronize(sl.done);
  if (sl.dev) (void)hipFree(sl.dev);
  if (sl.host) (void)hipHostFree(sl.host);
  sl.dev = sl.host = nullptr;
  size_t cap = std::max<size_t>(bytes * 2, 1 << 20);
  if (hipMalloc(&sl.dev, cap) != hipSuccess) return PACO_ERR_OUT_OF_MEMORY;
  if (hipHostMalloc(&sl.host, cap, hipHostMallocDefault) != hipSuccess) return PACO_ERR_OUT_OF_MEMORY;
  sl.cap = cap;
  (void)s;
  return PACO_OK;
}

paco_status grow_ws(paco_server s, uint64_t bytes) {
  if (bytes <= s->ws_bytes) return PACO_OK;
  // every launch that could touch the workspace is on the server's streams
  (void)hipStreamSynchronize(s->main);
  for (int g = 0; g < G_COUNT; ++g) (void)hipStreamSynchronize(s->gs[g]);
  if (s->ws) (void)hipFree(s->ws);
  s->ws = nullptr;
  s->ws_bytes = 0;
  uint64_t want = std::max<uint64_t>(bytes + bytes / 2, 64ull << 20);
  if (hipMalloc(&s->ws, want) != hipSuccess) return PACO_ERR_OUT_OF_MEMORY;
  s->ws_bytes = want;
  return PACO_OK;
}

// Launch one batch (dispatcher thread; no lock held).  Records b.ev.
paco_status launch_batch(paco_server s, Batch& b, std::vector<ReqState*>& rs, std::vector<paco_status>& rst) {
  const int nreq = (int)rs.size();
  rst.assign(nreq, PACO_OK);
  if (s->o.per_request) {
    for (int i = 0; i < nreq; ++i) {
      const ReqState* r = rs[i];
      paco_mm_desc d;
      memset(&d, 0, sizeof d);
      d.n = r->r.n; d.m = r->r.m; d.k = r->r.k; d.sr = r->r.sr;
      d.A = r->r.A; d.lda = r->r.lda; d.B = r->r.B; d.ldb = r->r.ldb; d.C = r->r.C; d.ldc = r->r.ldc;
      d.precision = r->r.precision;
      d.part = PACO_PART_PACO;
      paco_status st = paco_semiring_mm_ex(s->ctx, &d, nullptr);
      rst[i] = st;
      if (st != PACO_OK) b.ok = false;
    }
    return hipEventRecord(b.ev, s->main) == hipSuccess ? PACO_OK : PACO_ERR_HIP;
  }
  // ---- split over processors
  std::vector<BatchReq> br(nreq);
  for (int i = 0; i < nreq; ++i) {
    const paco_request& q = rs[i]->r;
    int prec = -1;
    if (q.sr == PACO_SR_PLUS_TIMES_F32) prec = q.precision == PACO_PREC_AUTO ? auto_precision(q.k) : (int)q.precision;
    br[i] = {q.n, q.m, q.k, (int)q.sr, prec};
  }
  BatchSplit bs = batch_partition(br, s->p);
  // ---- per group: problems, plan
  struct GroupPlan {
    std::vector<int> reqs;          // batch request index per local problem
    HostPlan h;
    int tile = 0;
    bool vec = true;
  } gp[G_COUNT];
  std::vector<int> local(nreq, -1);
  for (int i = 0; i < nreq; ++i) {
    int g = batch_group(br[i]);
    local[i] = (int)gp[g].reqs.size();
    gp[g].reqs.push_back(i);
  }
  int64_t temp_base = 0;
  for (int g = 0; g < G_COUNT; ++g) {
    if (gp[g].reqs.empty()) continue;
    std::vector<TaggedPiece> tp;
    std::vector<Piece> kpcs;
    std::vector<ProbGeom> geom;
    for (int i : gp[g].reqs) geom.push_back({br[i].n, rs[i]->mu, rs[i]->ku});
    for (const TaggedPiece& t : bs.pieces) {
      if (batch_group(br[t.prob]) != g) continue;
      TaggedPiece u = t;
      u.prob = local[t.prob];
      u.wg = t.wg - bs.g0[g];
      if (g == G_BOOL) {
        u.pc.m0 /= 32;
        u.pc.m1 = (u.pc.m1 + 31) / 32;
      }
      tp.push_back(u);
      kpcs.push_back(u.pc);
    }
    const int nwg = bs.g1[g] - bs.g0[g];
    gp[g].h = build_plan(tp, nwg, false, geom, temp_base);
    temp_base += (gp[g].h.temp_elems + 63) / 64 * 64;
    if (g != G_BOOL) {   // 128-bit operand loads (the boolean kernel has none)
      for (int i : gp[g].reqs) {
        const paco_request& q = rs[i]->r;
        if (!ring_vec_ok(q.A, q.lda ? q.lda : q.k, q.B, q.ldb ? q.ldb : q.m, q.m, q.k)) gp[g].vec = false;
      }
    }
    if (g <= G_RING_X6) {
      gp[g].tile = bs.tile[g];
    } else if (g == G_BOOL) {
      gp[g].tile = choose_bool_tile(kpcs);
      gp[g].vec = false;
    } else {
      gp[g].tile = choose_int_tile(kpcs);
      if (!gp[g].h.aligned4) gp[g].vec = false;
    }
  }
  paco_status st = grow_ws(s, (uint64_t)temp_base * 4);
  if (st != PACO_OK) return st;
  // ---- descriptor blob: per group problems | items | wg_off | tiles | srcs
  struct Off { size_t prob, items, wg, tiles, srcs; } off[G_COUNT];
  size_t tot = 0;
  auto take = [&](size_t bytes) {
    size_t o = tot;
    tot += (bytes + 255) & ~size_t(255);
    return o;
  };
  for (int g = 0; g < G_COUNT; ++g) {
    if (gp[g].reqs.empty()) continue;
    off[g].prob = take(sizeof(Problem) * gp[g].reqs.size());
    off[g].items = take(sizeof(WorkItem) * gp[g].h.items.size());
    off[g].wg = take(sizeof(int32_t) * gp[g].h.wg_off.size());
    off[g].tiles = take(sizeof(RedTile) * gp[g].h.tiles.size());
    off[g].srcs = take(sizeof(RedSrc) * gp[g].h.srcs.size());
  }
  Slot& sl = s->slots[s->next_slot];
  s->next_slot = (s->next_slot + 1) % kSlots;
  if (sl.used) (void)hipEventSynchronize(sl.done);   // its batch no longer reads the descriptors
  const bool zc = tot <= kZeroCopyBytes && sl.zdev;
  if (!zc && (st = grow_slot(s, sl, tot)) != PACO_OK) return st;
  char* hb = (char*)(zc ? sl.zhost : sl.host);
  for (int g = 0; g < G_COUNT; ++g) {
    if (gp[g].reqs.empty()) continue;
    Problem* pt = (Problem*)(hb + off[g].prob);
    for (size_t j = 0; j < gp[g].reqs.size(); ++j) {
      const ReqState* r = rs[gp[g].reqs[j]];
      Problem& P = pt[j];
      P.A = r->r.A; P.B = r->r.B; P.C = r->r.C;
      P.lda = r->r.lda ? r->r.lda : r->ku;
      P.ldb = r->r.ldb ? r->r.ldb : r->mu;
      P.ldc = r->r.ldc ? r->r.ldc : r->mu;
      P.n = (int32_t)r->r.n; P.m = (int32_t)r->r.m; P.k = (int32_t)r->r.k;
      P.accumulate = 0;
    }
    memcpy(hb + off[g].items, gp[g].h.items.data(), sizeof(WorkItem) * gp[g].h.items.size());
    memcpy(hb + off[g].wg, gp[g].h.wg_off.data(), sizeof(int32_t) * gp[g].h.wg_off.size());
    memcpy(hb + off[g].tiles, gp[g].h.tiles.data(), sizeof(RedTile) * gp[g].h.tiles.size());
    memcpy(hb + off[g].srcs, gp[g].h.srcs.data(), sizeof(RedSrc) * gp[g].h.srcs.size());
  }
  // Several kernel groups run side by side on their own streams, after the
  // descriptor copy and before the batch's completion event on the main
  // stream; a batch of one group (the usual case at light load) launches on
  // the main stream itself: each cross-stream event pair costs tens of
  // microseconds of host time, as much as the small requests' kernels.
  int ngroups = 0;
  for (int g = 0; g < G_COUNT; ++g) ngroups += gp[g].reqs.empty() ? 0 : 1;
  const bool single = ngroups == 1;
  hipError_t e = zc ? hipSuccess : hipMemcpyAsync(sl.dev, sl.host, tot, hipMemcpyHostToDevice, s->main);
  if (e == hipSuccess && !single) e = hipEventRecord(s->ready, s->main);
  char* db = (char*)(zc ? sl.zdev : sl.dev);
  for (int g = 0; g < G_COUNT && e == hipSuccess; ++g) {
    if (gp[g].reqs.empty()) continue;
    hipStream_t gsm = single ? s->main : s->gs[g];
    if (!single) e = hipStreamWaitEvent(gsm, s->ready, 0);
    if (e != hipSuccess) break;
    ProbRef pr;
    memset(&pr, 0, sizeof pr);
    pr.table = (const Problem*)(db + off[g].prob);
    pr.vec_ok = gp[g].vec ? 1 : 0;
    const WorkItem* items = (const WorkItem*)(db + off[g].items);
    const int32_t* wg = (const int32_t*)(db + off[g].wg);
    const int nwg = gp[g].h.nwg;
    if (g <= G_RING_X6) {
      const int prec = g == G_RING_FP32 ? PREC_FP32 : (g == G_RING_X3 ? PREC_BF16X3 : PREC_BF16X6);
      e = launch_ring(prec, gp[g].tile, pr, items, wg, nwg, 0, s->ws, gsm);
    } else if (g == G_BOOL) {
      e = launch_semiring_bool(gp[g].tile, pr, items, wg, nwg, 0, s->ws, gsm);
    } else {
      e = launch_semiring_int(g == G_MINPLUS ? SR_MINPLUS : SR_MAXPLUS, gp[g].tile, pr, items, wg, nwg, 0, s->ws,
                              gsm);
    }
    if (e == hipSuccess && !gp[g].h.tiles.empty()) {
      const int sr = g <= G_RING_X6 ? SR_RING : (g == G_BOOL ? SR_BOOL : (g == G_MINPLUS ? SR_MINPLUS : SR_MAXPLUS));
      e = launch_reduce(sr, pr, (const RedTile*)(db + off[g].tiles), (int)gp[g].h.tiles.size(),
                        (const RedSrc*)(db + off[g].srcs), s->ws, gsm, 1);
    }
    if (e == hipSuccess && !single) e = hipEventRecord(s->gdone[g], gsm);
    if (e == hipSuccess && !single) e = hipStreamWaitEvent(s->main, s->gdone[g], 0);
  }
  if (e == hipSuccess) e = hipEventRecord(b.ev, s->main);
  if (e == hipSuccess) e = hipEventRecord(sl.done, s->main);
  sl.used = true;
  if (e != hipSuccess) {
    set_err(s->ctx, std::string("server launch: ") + hipGetErrorString(e));
    return PACO_ERR_HIP;
  }
  return PACO_OK;
}

void dispatcher_main(paco_server s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  auto ready = [&] { return s->stop || (!s->queue.empty() && s->inflight.size() < 2); };
  while (true) {
    if (!ready() && s->o.spin_s > 0) {
      // poll before sleeping: a request arriving within spin_s is taken
      // without the wake-up of a sleeping thread
      const double until = paco_server_clock() + s->o.spin_s;
      do {
        lk.unlock();
        std::this_thread::yield();
        lk.lock();
      } while (!ready() && paco_server_clock() < until);
    }
    s->cv.wait(lk, ready);
    if (s->stop && s->queue.empty()) break;
    if (s->o.batch_window_s > 0 && !s->o.per_request) {
      const double first = s->reqs[s->queue.front()].res.arrival_s;
      while (!s->stop && (int)s->queue.size() < s->o.max_batch) {
        const double wait = first + s->o.batch_window_s - paco_server_clock();
        if (wait <= 0) break;
        s->cv.wait_for(lk, std::chrono::duration<double>(wait));
      }
    }
    // admit the head of the queue while the budget allows (FIFO)
    std::vector<uint64_t> take;
    std::vector<ReqState*> rs;
    const int cap = s->o.per_request ? 1 : s->o.max_batch;
    while (!s->queue.empty() && (int)take.size() < cap) {
      ReqState& r = s->reqs[s->queue.front()];
      if (s->bytes_in_flight + r.bytes > s->o.hbm_budget_bytes && !take.empty()) break;
      if (s->bytes_in_flight + r.bytes > s->o.hbm_budget_bytes && s->bytes_in_flight > 0) break;
      take.push_back(s->queue.front());
      rs.push_back(&r);
      s->bytes_in_flight += r.bytes;
      s->queue.pop_front();
    }
    if (take.empty()) {  // budget full: wait for a completion
      s->cv.wait(lk);
      continue;
    }
    Batch b;
    b.tickets = take;
    b.id = s->batch_counter++;
    (void)hipEventCreateWithFlags(&b.ev, hipEventDisableTiming);
    const double t = paco_server_clock();
    for (ReqState* r : rs) {
      r->res.launch_s = t;
      r->res.batch_id = b.id;
      r->res.batch_size = (int32_t)rs.size();
    }
    // request fields read while unlocked (r, mu, ku) are never written after submit
    std::vector<paco_status> rst;
    const bool inject = s->fail_next > 0;   // test hook: fail this batch before any launch
    if (inject) s->fail_next -= 1;
    lk.unlock();
    const paco_status st = inject ? PACO_ERR_INTERNAL : launch_batch(s, b, rs, rst);
    if (st != PACO_OK) {
      b.ok = false;
      (void)hipEventRecord(b.ev, s->main);
    }
    lk.lock();
    for (size_t i = 0; i < rs.size(); ++i)
      rs[i]->res.status = st != PACO_OK ? st : (i < rst.size() ? rst[i] : PACO_OK);
    s->inflight.push_back(b);
    s->batches += 1;
    s->batched_reqs += (int64_t)rs.size();
    s->cv.notify_all();
  }
  s->disp_done = true;
  s->cv.notify_all();
}

void completer_main(paco_server s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    s->cv.wait(lk, [&] { return s->disp_done || !s->inflight.empty(); });
    if (s->inflight.empty()) {
      if (s->disp_done) break;
      continue;
    }
    Batch b = s->inflight.front();
    lk.unlock();
    hipError_t e = hipEventSynchronize(b.ev);
    const double t = paco_server_clock();
    lk.lock();
    s->inflight.pop_front();
    for (uint64_t tk : b.tickets) {
      ReqState& r = s->reqs[tk];
      r.res.done_s = t;
      if (e != hipSuccess && r.res.status == PACO_OK) r.res.status = PACO_ERR_HIP;
      r.finished = true;
      s->bytes_in_flight -= r.bytes;
      s->pending -= 1;
      if (r.res.status == PACO_OK) {
        s->completed += 1;
        s->lat.add(r.res.done_s - r.res.arrival_s);
        s->ops += 2.0 * (double)r.r.n * (double)r.r.m * (double)r.r.k;
      } else {
        s->failed += 1;
      }
      // bounded retention: past kKeepFinished finished requests the oldest
      // unpolled one is forgotten
      s->finished_order.push_back(tk);
      if (s->finished_order.size() > kKeepFinished) {
        s->reqs.erase(s->finished_order.front());
        s->finished_order.pop_front();
      }
    }
    s->last_done = t;
    (void)hipEventDestroy(b.ev);
    s->cv.notify_all();
    s->cv_done.notify_all();
  }
}

}  // namespace

extern "C" paco_status paco_server_create(paco_ctx ctx, const paco_server_opts* opts, paco_server* out) {
  if (!ctx || !out) return PACO_ERR_INVALID_ARG;
  *out = nullptr;
  auto* s = new paco_server_s();
  if (opts) s->o = *opts;
  if (s->o.hbm_budget_bytes == 0) s->o.hbm_budget_bytes = 64ull << 30;
  if (s->o.max_batch <= 0) s->o.max_batch = 8192;
  if (s->o.p < 0 || s->o.batch_window_s < 0 || !(s->o.spin_s >= 0)) {
    delete s;
    return PACO_ERR_INVALID_ARG;
  }
  s->device = ctx->device;
  paco_status st = paco_create(&s->ctx, s->device, 0);
  if (st != PACO_OK) {
    delete s;
    return st;
  }
  s->p = s->o.p > 0 ? s->o.p : s->ctx->num_cus;
  // every request is planned anew (one-off shapes): the tile search of a
  // ring plan runs only where it may save 0.2 ms, in both modes
  s->ctx->search_min_gain = 2e-4;
  bool ok = hipStreamCreateWithFlags(&s->main, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&s->ready, hipEventDisableTiming) == hipSuccess;
  for (int g = 0; g < G_COUNT && ok; ++g)
    ok = hipStreamCreateWithFlags(&s->gs[g], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&s->gdone[g], hipEventDisableTiming) == hipSuccess;
  for (int i = 0; i < kSlots && ok; ++i) {
    Slot& sl = s->slots[i];
    ok = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess;
    // without a coherent mapped buffer the slot copies every blob instead
    if (ok && hipHostMalloc(&sl.zhost, kZeroCopyBytes, hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess &&
        hipHostGetDevicePointer(&sl.zdev, sl.zhost, 0) != hipSuccess) {
      (void)hipHostFree(sl.zhost);
      sl.zhost = sl.zdev = nullptr;
    }
    if (!sl.zhost) sl.zdev = nullptr;
    (void)hipGetLastError();   // a failed optional allocation is not the next call's error
  }
  if (!ok) {
    paco_server_destroy(s);
    return PACO_ERR_HIP;
  }
  s->ctx->stream = s->main;
  s->dispatcher = std::thread(dispatcher_main, s);
  s->completer = std::thread(completer_main, s);
  *out = s;
  return PACO_OK;
}

extern "C" paco_status paco_server_submit(paco_server s, const paco_request* r, uint64_t* ticket) {
  if (!s || !r || !ticket) return PACO_ERR_INVALID_ARG;
  if (r->n < 0 || r->m < 0 || r->k < 0 || r->n >= (1ll << 31) || r->m >= (1ll << 31) || r->k >= (1ll << 31) ||
      r->sr < PACO_SR_PLUS_TIMES_F32 || r->sr > PACO_SR_OR_AND_B1 || r->precision < PACO_PREC_FP32 ||
      r->precision > PACO_PREC_AUTO)
    return PACO_ERR_INVALID_ARG;
  ReqState st;
  st.r = *r;
  const bool is_bool = r->sr == PACO_SR_OR_AND_B1;
  st.mu = is_bool ? (r->m + 31) / 32 : r->m;
  st.ku = is_bool ? (r->k + 31) / 32 : r->k;
  if ((r->lda && r->lda < st.ku) || (r->ldb && r->ldb < st.mu) || (r->ldc && r->ldc < st.mu))
    return PACO_ERR_INVALID_ARG;
  // as paco_semiring_mm_ex: 32-bit offsets within a block of rows
  if ((r->lda ? r->lda : st.ku) >= (1ll << 22) || (r->ldb ? r->ldb : st.mu) >= (1ll << 22) ||
      (r->ldc ? r->ldc : st.mu) >= (1ll << 22))
    return PACO_ERR_UNSUPPORTED;
  if (r->n > 0 && r->m > 0 && (!r->C || (r->k > 0 && (!r->A || !r->B)))) return PACO_ERR_INVALID_ARG;
  if (r->k == 0) return PACO_ERR_UNSUPPORTED;   // the empty fold is a plain fill: use paco_semiring_mm
  st.bytes = req_bytes(*r, st.mu, st.ku);
  if (st.bytes > s->o.hbm_budget_bytes) return PACO_ERR_BUDGET;
  memset(&st.res, 0, sizeof st.res);
  const double now = paco_server_clock();
  st.res.arrival_s = r->arrival_s > 0 ? r->arrival_s : now;
  st.res.status = PACO_OK;
  st.res.precision = PACO_PREC_FP32;
  if (r->sr == PACO_SR_PLUS_TIMES_F32)
    st.res.precision = r->precision == PACO_PREC_AUTO ? (paco_precision)auto_precision(r->k) : r->precision;
  std::lock_guard<std::mutex> lk(s->mu);
  const uint64_t t = s->next_ticket++;
  if (s->first_arrival < 0 || st.res.arrival_s < s->first_arrival) s->first_arrival = st.res.arrival_s;
  s->reqs.emplace(t, st);
  s->queue.push_back(t);
  s->pending += 1;
  s->submitted += 1;
  *ticket = t;
  s->cv.notify_all();
  return PACO_OK;
}

extern "C" paco_status paco_server_poll(paco_server s, uint64_t ticket, int* done, paco_request_result* out) {
  if (!s || !done) return PACO_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return PACO_ERR_NOT_FOUND;
  *done = it->second.finished ? 1 : 0;
  if (out) *out = it->second.res;
  if (it->second.finished) s->reqs.erase(it);   // reported once, then forgotten
  return PACO_OK;
}

extern "C" paco_status paco_server_fail_batches(paco_server s, int32_t count) {
  if (!s || count < 0) return PACO_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  s->fail_next = count;
  return PACO_OK;
}

extern "C" paco_status paco_server_drain(paco_server s) {
  if (!s) return PACO_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->pending == 0; });
  return PACO_OK;
}

extern "C" paco_status paco_server_stats_get(paco_server s, paco_server_stats* out) {
  if (!s || !out) return PACO_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  memset(out, 0, sizeof *out);
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->failed = s->failed;
  out->batches = s->batches;
  out->mean_batch = s->batches ? (double)s->batched_reqs / (double)s->batches : 0.0;
  out->p50_s = s->lat.quantile(0.50);
  out->p99_s = s->lat.quantile(0.99);
  out->max_s = s->lat.maxv;
  out->span_s = s->first_arrival >= 0 ? s->last_done - s->first_arrival : 0.0;
  out->ops = s->ops;
  out->retained = (int64_t)s->reqs.size();
  out->bytes_in_flight = s->bytes_in_flight;
  return PACO_OK;
}

extern "C" paco_status paco_server_destroy(paco_server s) {
  if (!s) return PACO_ERR_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv.notify_all();
  }
  if (s->dispatcher.joinable()) s->dispatcher.join();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->cv.notify_all();
  }
  if (s->completer.joinable()) s->completer.join();
  (void)hipSetDevice(s->device);
  if (s->main) (void)hipStreamSynchronize(s->main);
  for (int g = 0; g < G_COUNT; ++g) {
    if (s->gs[g]) {
      (void)hipStreamSynchronize(s->gs[g]);
      (void)hipStreamDestroy(s->gs[g]);
    }
    if (s->gdone[g]) (void)hipEventDestroy(s->gdone[g]);
  }
  for (int i = 0; i < kSlots; ++i) {
    if (s->slots[i].dev) (void)hipFree(s->slots[i].dev);
    if (s->slots[i].host) (void)hipHostFree(s->slots[i].host);
    if (s->slots[i].zhost) (void)hipHostFree(s->slots[i].zhost);
    if (s->slots[i].done) (void)hipEventDestroy(s->slots[i].done);
  }
  if (s->ready) (void)hipEventDestroy(s->ready);
  if (s->ws) (void)hipFree(s->ws);
  if (s->ctx) {
    s->ctx->stream = nullptr;
    paco_destroy(s->ctx);
  }
  if (s->main) (void)hipStreamDestroy(s->main);
  delete s;
  return PACO_OK;
}

extern "C" paco_status paco_batch_partition(const paco_request* reqs, int32_t nreq, int32_t p, paco_piece* out,
                                            int32_t* req_of_piece, int64_t cap, int64_t* n_out) {
  if (!reqs || nreq < 0 || p < 1 || !n_out || (cap > 0 && (!out || !req_of_piece))) return PACO_ERR_INVALID_ARG;
  std::vector<BatchReq> br(nreq);
  for (int i = 0; i < nreq; ++i) {
    const paco_request& q = reqs[i];
    if (q.n < 0 || q.m < 0 || q.k < 0 || q.sr < PACO_SR_PLUS_TIMES_F32 || q.sr > PACO_SR_OR_AND_B1)
      return PACO_ERR_INVALID_ARG;
    int prec = -1;
    if (q.sr == PACO_SR_PLUS_TIMES_F32) prec = q.precision == PACO_PREC_AUTO ? auto_precision(q.k) : (int)q.precision;
    br[i] = {q.n, q.m, q.k, (int)q.sr, prec};
  }
  BatchSplit bs = batch_partition(br, p);
  *n_out = (int64_t)bs.pieces.size();
  for (int64_t i = 0; i < std::min<int64_t>(cap, (int64_t)bs.pieces.size()); ++i) {
    const TaggedPiece& t = bs.pieces[i];
    out[i].n0 = t.pc.n0; out[i].n1 = t.pc.n1;
    out[i].m0 = t.pc.m0; out[i].m1 = t.pc.m1;
    out[i].k0 = t.pc.k0; out[i].k1 = t.pc.k1;
    out[i].proc = t.wg;
    out[i].temp = t.pc.k0 > 0 ? 1 : 0;
    out[i].round = 0;
    out[i].depth = t.pc.depth;
    req_of_piece[i] = t.prob;
  }
  return PACO_OK;
}

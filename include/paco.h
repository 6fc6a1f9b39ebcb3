/*
 * paco.h -- C ABI of libpaco: PACO-partitioned semiring matrix multiplication
 * and Strassen's algorithm on one AMD Instinct MI355X (gfx950).
 *
 * Method: Tang & Gao, "Balanced Partitioning of Several Cache-Oblivious
 * Algorithms" (arXiv 2011.01441), sections "PACO MM" (problem statement,
 * cuboid view, MM-1-Piece), "Extension to Heterogeneous Computing System"
 * and "PACO Strassen".
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Matrices are dense and row-major.  A is n-by-k, B is k-by-m, C is
 *    n-by-m (the problem statement's orientation), each with a leading
 *    dimension (elements between rows) of at least its column count and
 *    below 2^22 (PACO_ERR_UNSUPPORTED otherwise: the kernels address a
 *    block of rows with 32-bit offsets from a 64-bit row base).
 *  - Operand and result pointers A, B, C are DEVICE pointers owned by the
 *    caller.  The library never frees them and keeps no reference past the
 *    call.  Calls are asynchronous on the context's stream: keep the buffers
 *    alive and unmodified until that stream has been synchronised.
 *  - Boolean matrices are bit-packed: row r of an R-by-W bit matrix is
 *    ceil(W/32) uint32 words, bit w lives in bit (w % 32) of word (w / 32),
 *    least significant bit first; padding bits of inputs must be 0 and
 *    padding bits of C are written 0.  Leading dimensions count words.
 *  - Semiring constants (the paper leaves them open; these are this
 *    library's definitions):
 *      (min,+) int32: zero INF = 2^30; product min(a+b, INF); valid entries
 *                     lie in [0, 2^30].
 *      (max,+) int32: zero NEG_INF = -2^30; product a+b, or NEG_INF when
 *                     either factor is NEG_INF; finite entries lie in
 *                     [-2^28, 2^28].
 *      boolean      : OR of ANDs.
 *      (+,x) float32: IEEE float32 results; see paco_precision.
 *    Entries outside these domains give unspecified (but memory-safe)
 *    results.
 *  - Errors are returned as paco_status; nothing aborts or throws across
 *    the ABI.  A per-context message is kept for the last failure.
 *  - One context per host thread.  Workspace (temporary faces for k-cuts,
 *    Strassen temporaries, piece descriptors) is owned by the context,
 *    grows on demand and is capped by the budget given at creation.
 */
#ifndef PACO_H
#define PACO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The enumerations below are int32 in the ABI.  C++ callers and the library
 * itself see them with that fixed underlying type, so that any int32 a C
 * caller passes is a value the entry points can test and reject with
 * PACO_ERR_INVALID_ARG (an out-of-range value of an enumeration without one
 * is undefined in C++). */
#ifdef __cplusplus
#define PACO_ENUM_INT32 : int32_t
#else
#define PACO_ENUM_INT32
#endif

typedef enum paco_status PACO_ENUM_INT32 {
  PACO_OK = 0,
  PACO_ERR_INVALID_ARG = 1,   /* null pointer, negative size, bad enum, bad ld */
  PACO_ERR_UNSUPPORTED = 2,   /* e.g. Strassen on a non-ring semiring */
  PACO_ERR_OUT_OF_MEMORY = 3, /* a device allocation failed */
  PACO_ERR_BUDGET = 4,        /* workspace or admission budget exceeded */
  PACO_ERR_HIP = 5,           /* a HIP runtime call failed */
  PACO_ERR_INTERNAL = 6,
  PACO_ERR_NOT_FOUND = 7      /* unknown server ticket */
} paco_status;

typedef enum paco_semiring PACO_ENUM_INT32 {
  PACO_SR_PLUS_TIMES_F32 = 0, /* (+,x) ring on float32 */
  PACO_SR_MIN_PLUS_I32 = 1,   /* tropical (min,+) on int32 */
  PACO_SR_MAX_PLUS_I32 = 2,   /* (max,+) on int32 */
  PACO_SR_OR_AND_B1 = 3       /* boolean, bit-packed uint32 words */
} paco_semiring;

/* Arithmetic of the (+,x) ring path.
 *  FP32   : float32 matrix-core products with float32 accumulation.
 *  BF16X3 : each float32 operand x is split into hi = bf16(x) and
 *           lo = bf16(x - hi) (round to nearest even); the product is
 *           hi*hi' + hi*lo' + lo*hi' on bf16 matrix cores with float32
 *           accumulation (split-precision method of Henry, Tang & Heinecke,
 *           2019).
 *  BF16X6 : three-way split hi, mid, lo and the six products whose
 *           combined significance reaches float32 (hi*hi', hi*mid',
 *           mid*hi', mid*mid', hi*lo', lo*hi').
 *  AUTO   : BF16X3 when its predicted componentwise error at this k is at
 *           most 2^-21, BF16X6 otherwise.  The prediction is for entries of
 *           similar magnitude (errors of many terms averaging out); where a
 *           few large terms dominate each output, as with entries spread
 *           over many decades, BF16X3 can reach about 2^-15 and BF16X6
 *           should be asked for explicitly.
 * Integer and boolean semirings ignore this field. */
typedef enum paco_precision PACO_ENUM_INT32 {
  PACO_PREC_FP32 = 0,
  PACO_PREC_BF16X3 = 1,
  PACO_PREC_BF16X6 = 2,
  PACO_PREC_AUTO = 3
} paco_precision;

/* How the n-by-m-by-k iteration cuboid is split over workgroups.
 *  PACO : MM-1-Piece (section "PACO MM", corollary mm-1-piece): recursive
 *         cuts of the longest dimension of a same-sized virtual cuboid in
 *         the ratio floor(p/2):ceil(p/2), one cuboid per processor (one
 *         persistent workgroup per compute unit).
 *  GRID : the baseline the paper's experiments compare against in spirit:
 *         the same microkernel on a plain grid of output tiles with a
 *         split-k factor chosen by the autotuner. */
typedef enum paco_part_mode PACO_ENUM_INT32 {
  PACO_PART_PACO = 0,   /* MM-1-Piece: one piece per processor */
  PACO_PART_GRID = 1,   /* plain output-tile grid with split-k (baseline) */
  PACO_PART_MULTI = 2   /* multi-piece pruned BFS (theorem mm): every cut
                           halves a cuboid; a depth with >= p unassigned
                           cuboids hands p of them out; at most 4 rounds,
                           then the rest round-robin */
} paco_part_mode;

typedef struct paco_ctx_s* paco_ctx;

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device`.  workspace_budget_bytes caps the
 * device workspace the context may hold (0 = 64 GiB).  The context creates
 * no stream of its own; it launches on the stream set by paco_set_stream
 * (initially the null stream).  It caches one plan (host work lists and
 * their device tables) per call shape, up to 512: a call that needs a new
 * plan when 512 are held first synchronises the device and drops them all,
 * after which graphs captured earlier refuse to replay (PACO_ERR_INVALID_ARG
 * from paco_graph_launch, as after a workspace change). */
paco_status paco_create(paco_ctx* out, int device, uint64_t workspace_budget_bytes);
paco_status paco_destroy(paco_ctx ctx);
/* `stream` is a hipStream_t passed as an opaque pointer.  Every call of a
 * context shares its workspace (temporary faces, Strassen temporaries), so
 * when the stream changes, the new stream first waits (an event, no host
 * synchronisation) for everything the context launched on the previous
 * one: calls made through one context run in the order they were made,
 * whichever streams they were given. */
paco_status paco_set_stream(paco_ctx ctx, void* stream);
/* The device's compute units.  The default processor count of a PACO call
 * is this times the number of workgroups of the chosen kernel that fit on
 * one compute unit at once (1 for the matrix-core ring kernel, 2-4 for the
 * VALU kernels); paco_mm_result.p reports the value used. */
int paco_num_cus(paco_ctx ctx);
/* Device-side balance record (section "PACO Design and Analysis": every
 * processor should finish at the same time).  With `stamps` set (a DEVICE
 * buffer of 4 * capacity uint64 words, owned by the caller), each later
 * semiring MM call of this context (paco_semiring_mm, _ex, _noalloc) has
 * the workgroup standing for processor q < capacity write, at
 * stamps[4q .. 4q+3]: the start and the end of its work, on the device's
 * 100 MHz real-time counter, and the XCC_ID and HW_ID hardware registers of
 * where it ran (processors of a GRID call are its output tiles).  Slots of
 * processors the call does not have keep their old contents.  Each kernel
 * adds one barrier per processor while it is set.  NULL (capacity 0) turns
 * it off.  paco_strassen_mm records its batched leaf product; the pruned-BFS
 * Strassen and server calls record nothing. */
paco_status paco_set_piece_stamps(paco_ctx ctx, void* stamps, int32_t capacity);
const char* paco_status_string(paco_status s);
const char* paco_last_error(paco_ctx ctx);

/* --------------------------------------------------------- semiring MM */

/* C = A (x) B over semiring `sr` (section "PACO MM", problem statement),
 * dense operands with lda = k, ldb = m, ldc = m (words for boolean),
 * PACO partition over all compute units, precision AUTO for the ring.
 * n = 0 or m = 0 is a no-op; k = 0 writes the semiring zero into C. */
paco_status paco_semiring_mm(paco_ctx ctx, int64_t n, int64_t m, int64_t k,
                             paco_semiring sr, const void* A, const void* B, void* C);

typedef struct paco_mm_desc {
  int64_t n, m, k;
  paco_semiring sr;
  const void* A; int64_t lda;   /* 0 = dense default */
  const void* B; int64_t ldb;
  void* C;       int64_t ldc;
  int32_t accumulate;           /* nonzero: C <- C (+) A (x) B */
  paco_precision precision;     /* ring only */
  paco_part_mode part;
  int32_t p;                    /* processors (workgroups); 0 = compute units
                                   x resident workgroups per compute unit */
  int32_t grid_split_k;         /* GRID mode split-k; 0 = autotuned */
  int32_t verify_rows;          /* >0: float64 check of this many sampled
                                   rows on the GPU (ring only); the call
                                   then synchronises the stream */
  uint64_t verify_seed;
  double kcut_cost;             /* PACO mode: when the longest dimension of
                                   the virtual cuboid is chosen, k counts as
                                   k / kcut_cost (1 = the paper's rule; a
                                   k-cut costs a temporary face written and
                                   read back); 0 = library default: 16
                                   for the ring, chosen among 1, 4, 16 and
                                   64 with the tile and p for the others;
                                   values below 1, or not finite, are
                                   PACO_ERR_INVALID_ARG */
  const double* weights;        /* NULL, or p positive processor throughputs
                                   (host memory, read during the call): PACO
                                   mode with an explicit p cuts each cuboid
                                   in the ratio of the summed throughputs of
                                   the two halves of the processor list (the
                                   heterogeneous variant of the experiments
                                   section), e.g. from paco_calibrate */
} paco_mm_desc;

typedef struct paco_mm_result {
  paco_precision precision;     /* precision actually used (ring) */
  int32_t p;                    /* processors used */
  int32_t n_pieces;             /* non-empty pieces */
  int64_t max_piece_volume, min_piece_volume;  /* n'*m'*k' over non-empty pieces */
  int64_t temp_elems;           /* temporary-face elements for k-cuts */
  int32_t n_kcuts;              /* pieces writing a temporary face */
  double verify_max_rel;        /* max |C-C64| / (|A||B|) over sampled rows, -1 if not verified */
  double verify_max_abs;        /* max |C-C64| over sampled rows */
  double kcut_cost;             /* k-cut cost the PACO partition used */
} paco_mm_result;

/* Extended form: explicit leading dimensions, accumulation, precision,
 * partition mode and processor count.  `out` may be NULL.
 *
 * Environment overrides, read when a plan is built (for experiments and
 * the tile-grid baseline's autotuning; each value is part of the plan-cache
 * key, so changing it builds a new plan):
 *   PACO_KCUT_COST  k-cut cost used when the caller gives 0 (values below 1
 *                   count as 1);
 *   PACO_RING_TILE, PACO_INT_TILE, PACO_BOOL_TILE
 *                   index of the tile shape of the ring, (min,+)/(max,+) or
 *                   boolean kernel, overriding the chosen one (out-of-range
 *                   values are ignored);
 *   PACO_FUSE_FOLD  1: the product kernel folds the temporary faces of
 *                   k-cuts itself (the last piece to finish a reduction
 *                   cell folds it, same order and results), 2: only when
 *                   every cell is small, 0 (default): a second launch folds
 *                   them (measured faster on this device). */
paco_status paco_semiring_mm_ex(paco_ctx ctx, const paco_mm_desc* d, paco_mm_result* out);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * call as paco_semiring_mm_ex (same plan, same kernels, bit-identical
 * results), except that it calls no hipMalloc, hipFree or other allocating
 * routine: the plan's device tables and the temporary faces of its k-cuts
 * are placed in one fixed device array of PACO_NOALLOC_SCRATCH_BYTES
 * (64 MiB), which every device the library runs on holds from the first
 * paco_create on that device until the process ends.  Each call first
 * copies the plan's tables (kept in host memory, cached per shape by the
 * context) into that array on the context's stream, then launches.
 *  - A plan whose tables and faces exceed the array returns PACO_ERR_BUDGET
 *    without launching anything (raise kcut_cost for fewer k-cuts).
 *  - verify_rows > 0 returns PACO_ERR_UNSUPPORTED.
 *  - Every call on one device shares that device's array, and the array
 *    keeps the last call's contents: calls that overlap on one device
 *    (different streams or contexts without ordering between them) race and
 *    give wrong results.  Calls on one stream are ordered. */
#define PACO_NOALLOC_SCRATCH_BYTES (64ull << 20)
paco_status paco_semiring_mm_noalloc(paco_ctx ctx, const paco_mm_desc* d, paco_mm_result* out);
/* PACO_NOALLOC_SCRATCH_BYTES as the library was built with. */
uint64_t paco_noalloc_scratch_bytes(void);

/* Host-only argument check of a descriptor: the status paco_semiring_mm_ex
 * would return for it before touching the device (PACO_OK, or
 * PACO_ERR_INVALID_ARG / PACO_ERR_UNSUPPORTED as documented above).
 * Operand pointers are only tested for NULL. */
paco_status paco_mm_validate(const paco_mm_desc* d);

/* Measure the throughput of p processors (workgroups of one launch, p a
 * multiple of 8, at most 8 x compute units) for the heterogeneous split
 * (section "Extension to Heterogeneous Computing System"): all of them run
 * the same matrix-core chain at once, after an untimed run of the same
 * length so that clocks and power settle; each processor's rate is that of
 * its XCD (processors q of XCD q / (p/8), as PACO launches place them),
 * in bf16 TFLOP/s.  iters = 0: about 50 ms per run.  Synchronous. */
paco_status paco_calibrate(paco_ctx ctx, int32_t p, int32_t iters, double* rates);

/* Measured peaks of this device, for the rooflines' denominators:
 *   PACO_PEAK_MFMA_BF16  bf16 matrix-core products (32x32x16), TFLOP/s
 *   PACO_PEAK_VALU_I32   u32 add and min vector instructions, T lane-instr/s
 *   PACO_PEAK_VALU_F32   fp32 fused multiply-adds (unpacked), TFLOP/s
 *   PACO_PEAK_HBM_COPY   1 GiB device-to-device copy, GB/s (read + written)
 * Each probe runs twice on the context stream (the first untimed) with four
 * workgroups per compute unit and is timed between events; it allocates
 * and frees its own buffers (2 GiB for the copy).  Synchronous.  Unknown
 * kind: PACO_ERR_INVALID_ARG. */
typedef enum PACO_ENUM_INT32 {
  PACO_PEAK_MFMA_BF16 = 0,
  PACO_PEAK_VALU_I32 = 1,
  PACO_PEAK_VALU_F32 = 2,
  PACO_PEAK_HBM_COPY = 3
} paco_peak_kind;
paco_status paco_peak(paco_ctx ctx, paco_peak_kind kind, double* rate);

/* Keep p processor throughputs in the context (copied): from then on ring
 * calls in PACO mode that leave p and weights at 0 run on p processors with
 * the heterogeneous split.  p = 0 or weights = NULL clears them.  p must be
 * the compute-unit count (the ring kernel holds one workgroup per unit). */
paco_status paco_set_processor_weights(paco_ctx ctx, int32_t p, const double* weights);

/* ------------------------------------------------------------- Strassen */

/* C = A B for n-by-n float32 matrices (section "PACO Strassen"): `levels`
 * levels of Strassen's 7-product recursion (1-based S1..S7, T1..T7,
 * M_r = S_r T_r, quadrant sums of M), all 7^levels leaf products run as one
 * PACO-partitioned batch on the ring kernel at precision `leaf`.
 * levels in [0, 3]; n must be divisible by 2^levels (else UNSUPPORTED).
 * A, B, C dense (ld = n), device pointers. */
paco_status paco_strassen_mm(paco_ctx ctx, int64_t n, const float* A, const float* B,
                             float* C, int levels, paco_precision leaf);

/* PACO Strassen with the pruned breadth-first schedule of section "PACO
 * Strassen" (and its corollary Strassen-Const-Pieces).  The 7-way recursion
 * tree is expanded depth by depth, with every S, T and M of a depth held in
 * temporary space.  At a depth with N >= p unassigned nodes, floor(N/p)*p of
 * them (the first in breadth-first order) are handed out, node i to
 * processor i mod p, and the rest are divided again.  After `gamma`
 * super-rounds (0: no limit), or when nodes would become smaller than `base`
 * or of odd size, all remaining nodes are handed out round-robin.
 *
 * A processor here is a group of num_cus/p consecutive compute units (p = 8:
 * one XCD with its own L2, the private cache of the paper's processor).  It
 * runs each of its nodes as a classic product on the matrix-core kernel,
 * split over the group's compute units by MM-1-Piece.  The paper runs an
 * assigned node with sequential Strassen on one processor; here the node's
 * size is the recursion cutoff.  All assigned nodes of all depths run in one
 * persistent launch; pre-additions run before it and combines after it, both
 * one depth at a time (the top min(first assigning depth, 3) levels fused).
 *
 * A, B, C: dense n-by-n float32 device pointers.  p in [1, compute units]
 * (0 = compute units / 32, one per XCD).  base >= 1 (0 = 256).  leaf: ring
 * precision of the node products (AUTO: bf16x3 when the first assigned
 * nodes are at least 1024 wide, else bf16x6). */
typedef struct paco_strassen_desc {
  int64_t n;
  const float* A;
  const float* B;
  float* C;
  int32_t p;
  int32_t gamma;
  int64_t base;
  paco_precision leaf;
} paco_strassen_desc;

typedef struct paco_strassen_result {
  int32_t p;                 /* processors (groups of compute units) */
  int32_t super_rounds;      /* depths that handed out floor(N/p)*p nodes */
  int32_t max_depth;         /* deepest depth with assigned nodes */
  int64_t nodes;             /* nodes handed out */
  double max_work, min_work; /* per processor: sum of node n'^3 */
  uint64_t temp_bytes;       /* S, T, M of all depths */
  paco_precision leaf;
} paco_strassen_result;

paco_status paco_strassen_pbfs(paco_ctx ctx, const paco_strassen_desc* d, paco_strassen_result* out);

/* ---------------------------------------------------------- 1D problem */

/* The 1D problem (section "PACO 1D", equation (1D)), also known as least
 * weight subsequence: given D[0], D[j] = min over 0 <= i < j of
 * D[i] + w(i, j) for j = 1..n, with a weight function that needs no memory:
 *   PACO_W_AFFINE  w(i, j) = a + b (j - i)                 (a, b >= 0)
 *   PACO_W_HASH    w(i, j) = a + (fmix32(key) mod 2^b),   0 <= b <= 29,
 *                  key = (i * 0x9E3779B9 + j) mod 2^32, XOR seed, fmix32
 *                  MurmurHash3's 32-bit finaliser.
 * Values are integers with INF = 2^30 as "no path" and saturating sums.
 * The weights must stay within INF: a + b n <= 2^30 (affine) or
 * a + 2^b <= 2^30 (hash); otherwise PACO_ERR_UNSUPPORTED.
 *
 * The recursion of the section: the positions [0, n] split in halves (cut
 * points on multiples of 64), the left half is solved, its outputs update
 * the right half's (a square of inputs by outputs), then the right half is
 * solved; halves of at most `base` positions are base triangles run by one
 * workgroup.  part = PACO_PART_PACO cuts each square over
 * min(p, area / min_piece) processors (at least 1) by the ratio rule of
 * MM-1-Piece on its longer side (outputs on ties); pieces whose inputs were
 * cut combine with atomic minima.  PACO_PART_GRID (baseline) splits the
 * outputs only, into at most that many strips of at least 64.
 *
 * D: device array of n + 1 int32, D[0] read (in [0, 2^30]; outside reads as
 * INF), D[1..n] written.  Asynchronous on the context stream; the plan is
 * cached per (n, part, p, base, min_piece).  Calls on one context must not
 * overlap (each plan keeps its own launch counters). */
typedef enum PACO_ENUM_INT32 { PACO_W_AFFINE = 0, PACO_W_HASH = 1 } paco_w_kind;

typedef struct paco_dp1d_desc {
  int64_t n;
  int32_t w_kind;      /* paco_w_kind */
  int32_t a;           /* weight offset */
  int32_t b;           /* affine slope, or hash bits */
  uint32_t seed;       /* hash seed */
  int32_t part;        /* PACO_PART_PACO or PACO_PART_GRID */
  int32_t p;           /* processors; 0: 4 per compute unit */
  int32_t base;        /* longest base triangle, 64..1024; 0: 512 */
  int32_t min_piece;   /* least pairs per piece; 0: 65536 */
  int32_t* D;
} paco_dp1d_desc;

typedef struct paco_dp1d_result {
  int32_t p;             /* processors used */
  int32_t launches;      /* kernel launches of one call */
  int64_t triangles;     /* base triangles */
  int64_t squares;       /* external updates */
  int64_t pieces;        /* pieces over all squares */
  int32_t max_pieces;    /* most pieces of one square */
  int32_t atomic_pieces; /* pieces whose inputs were cut, over all squares */
} paco_dp1d_result;

paco_status paco_dp1d(paco_ctx ctx, const paco_dp1d_desc* desc, paco_dp1d_result* result);

/* Host-only: the plan paco_dp1d launches for (n, part, p, base, min_piece)
 * (all explicit here: p >= 1, base in 64..1024, min_piece >= 1).  info[0]
 * and info[1] give the capacities of `squares` and `pieces` on input (when
 * they are non-NULL) and their counts on output; info[2] = length of the
 * first base triangle [0, info[2]); info[3] = number of base triangles.
 *   squares: 8 int64 each (lo, mid, hi, first piece, piece count, lo and
 *            length of the base triangle that follows, and how many of the
 *            first pieces reach into it), in launch order;
 *   pieces : 5 int64 each (i0, i1, j0, j1, inputs cut). */
paco_status paco_dp1d_plan_export(int64_t n, int32_t part, int32_t p, int32_t base, int32_t min_piece,
                                  int64_t* info, int64_t* squares, int64_t* pieces);

/* --------------------------------------------------------- GAP problem */

/* The GAP problem (section "PACO GAP", equation (gap)): edit distance with
 * gaps.  On the (m+1) x (n+1) grid D (row-major, leading dimension ldd),
 * D[0][0] given and, for every other cell,
 *   D[i][j] = min( D[i-1][j-1] + s(i, j)              (i, j >= 1),
 *                  min over q < j of D[i][q] + w(q, j),
 *                  min over p < i of D[p][j] + w'(p, i) ),
 * saturated at INF = 2^30.  w (w_row) and w' (w_col) are weight functions of
 * the 1D problem's families (paco_w_kind; affine a + b (to - from) with
 * a + b side <= 2^30, or hashed with b <= 29 bits).  s is the substitution
 * cost of two symbol sequences over an alphabet of 2^s_bits symbols,
 * x_i = fmix32(i XOR s_seed_x) mod 2^s_bits, y_j = fmix32(j XOR s_seed_y)
 * mod 2^s_bits: s_match when x_i = y_j, else s_mismatch (both <= 2^30).
 *
 * The recursion of the section: quadrants; the rows of a finished top-left
 * quadrant update the top-right one, its columns the bottom-left one
 * (external updates, cubes of batch x inputs x outputs), down to base blocks
 * of at most 64 x 64 solved by one workgroup.  Independent subproblems share
 * launches.  part = PACO_PART_PACO cuts every cube among its volume share of
 * p processors (at least 1, at most volume / min_piece) into slabs of whole
 * batch rows, the section's rule, so each piece updates outputs of its own
 * (a batch shorter than the share also cuts the outputs, in multiples of
 * 64); PACO_PART_GRID (baseline) tiles every cube into 16 batch rows x 256
 * outputs, whatever p.
 *
 * D: device array, caller-owned; D[0][0] read (values outside [0, 2^30]
 * read as INF), every cell written.  The context keeps a transposed copy of
 * the grid ((n+1) x (m+1) rounded up to 64, counted against the budget:
 * PACO_ERR_BUDGET when it does not fit).  Asynchronous on the context
 * stream; the plan is cached per (m, n, part, p, min_piece). */
typedef struct paco_weight {
  int32_t kind;    /* paco_w_kind */
  int32_t a, b;    /* offset; affine slope or hash bits */
  uint32_t seed;   /* hash seed */
} paco_weight;

typedef struct paco_gap_desc {
  int64_t m, n;              /* grid (m+1) x (n+1) */
  paco_weight w_row;         /* w(q, j), gaps along a row */
  paco_weight w_col;         /* w'(p, i), gaps along a column */
  int32_t s_match, s_mismatch, s_bits;
  uint32_t s_seed_x, s_seed_y;
  int32_t part;              /* PACO_PART_PACO or PACO_PART_GRID */
  int32_t p;                 /* processors; 0: 4 per compute unit */
  int32_t min_piece;         /* least pairs per piece; 0: 16384 */
  int32_t* D;
  int64_t ldd;               /* >= n + 1 */
} paco_gap_desc;

typedef struct paco_gap_result {
  int32_t p;                 /* processors used */
  int32_t launches;          /* kernel launches of one call */
  int64_t base_blocks;       /* base blocks */
  int64_t cubes;             /* external updates */
  int64_t pieces;            /* pieces over all cubes */
} paco_gap_result;

paco_status paco_gap(paco_ctx ctx, const paco_gap_desc* desc, paco_gap_result* result);

/* Host-only: the plan paco_gap launches for (m, n, part, p, min_piece), all
 * explicit (p >= 1, min_piece >= 1).  info[0..2] give the capacities of
 * `launches`, `blocks` and `pieces` on input (when non-NULL) and their counts
 * on output; info[3] = number of cubes.
 *   launches: 3 int64 each (1 for base blocks / 0 for cubes, first entry,
 *             count), in order after the fill;
 *   blocks  : 4 int64 each (r0, r1, c0, c1);
 *   pieces  : 7 int64 each (column-gap flag, batch t0, t1, inputs x0, x1,
 *             outputs o0, o1). */
paco_status paco_gap_plan_export(int64_t m, int64_t n, int32_t part, int32_t p, int32_t min_piece, int64_t* info,
                                 int64_t* launches, int64_t* blocks, int64_t* pieces);

/* ------------------------------------------------------------- tuning */

/* Measured choice for one shape.  `d` is a default PACO call (part PACO,
 * p, kcut_cost, weights, verify_rows and accumulate all 0) on real
 * operands; the tuner runs it and its alternatives -- ring: MM-1-Piece and
 * multi-piece, k-cut cost 1/4/16/64, each ring tile; VALU semirings: each
 * tile at CUs x its resident workgroups and 4 times that, k-cut cost
 * 1/16/64 -- times each on the context stream (C is overwritten), and keeps
 * the fastest in the context if it beats the default.  Later calls of the
 * same (semiring, n, m, k, precision) with default options use it.
 * Synchronous; candidates that fail (e.g. over the workspace budget) are
 * skipped.  paco_tune_clear forgets every choice. */
typedef struct paco_tune_result {
  int32_t tuned;             /* 1: a candidate beat the default and was kept */
  paco_part_mode part;
  int32_t p, tile, weighted; /* tile: index of the kernel's tile list */
  double kcut_cost;
  double best_ms, default_ms;
  int32_t candidates;        /* candidates timed */
} paco_tune_result;

paco_status paco_tune(paco_ctx ctx, const paco_mm_desc* d, paco_tune_result* out);
paco_status paco_tune_clear(paco_ctx ctx);

/* ------------------------------------------------------------ hipGraphs */

/* A call captured once and replayed.  paco_graph_create runs the call
 * eagerly on the context stream (building and uploading its plan, sizing
 * the workspace), waits for it, then records `repeat` (1..4096)
 * back-to-back runs of the call's kernel launches into a hipGraph on a
 * private stream and instantiates it.  Each graph launch carries a fixed
 * cost (measured 5-100 us on ROCm 7.2), so capturing several runs pays off
 * for short calls.
 * paco_graph_launch replays those launches on `stream` (a hipStream_t as an
 * opaque pointer; NULL = the context stream) with the operand pointers and
 * sizes of the capture, reading whatever the buffers hold at replay time.
 * The launches point into the context's workspace: a later call that
 * grows it makes earlier graphs stale, and paco_graph_launch then returns
 * PACO_ERR_INVALID_ARG instead of replaying (create graphs after the calls
 * that need the most workspace, or use one context per graph).  The
 * operand buffers must outlive the graph.  verify_rows must be 0.  Replays of one graph
 * on one stream are ordered; replays that overlap with other calls on the
 * same context race on its workspace. */
typedef struct paco_graph_s* paco_graph;
paco_status paco_graph_create(paco_ctx ctx, const paco_mm_desc* d, int32_t repeat, paco_graph* out);
paco_status paco_graph_create_strassen(paco_ctx ctx, const paco_strassen_desc* d, int32_t repeat,
                                       paco_graph* out);
paco_status paco_graph_launch(paco_graph g, void* stream);
paco_status paco_graph_destroy(paco_graph g);

/* Host-only: the schedule paco_strassen_pbfs runs.  levels[i] describes
 * depth i (the node dimension h, the nodes of the depth, how many were
 * handed out, whether the depth was a super-round); work_classic[j] and
 * work_strassen[j] (optional, p entries) are processor j's sum of h^3 and of
 * h^log2(7) over its nodes.  Call with cap = 0 to get *n_levels. */
typedef struct paco_strassen_level {
  int32_t depth, super_round;
  int64_t h, nodes, assigned;
} paco_strassen_level;

paco_status paco_strassen_schedule(int64_t n, int32_t p, int32_t gamma, int64_t base,
                                   paco_strassen_level* levels, int32_t cap, int32_t* n_levels,
                                   double* work_classic, double* work_strassen);

/* ----------------------------------------------------- float64 checker */

/* For `nrows` rows listed in the device array `rows` (int64), compute on
 * the GPU in float64 C64 = A B and S = |A||B| and reduce
 *   out[0] = max |C - C64| / S   (componentwise, entries with S = 0 skipped)
 *   out[1] = max |C - C64|
 *   out[2] = sum (C - C64)^2,  out[3] = sum C64^2
 * into the host array out[4].  A NaN or infinite entry of C in a sampled
 * row counts as an infinite error (out[0] = out[1] = +infinity).  Dense float32 A (n-by-k), B (k-by-m),
 * C (n-by-m).  Synchronises the context stream. */
paco_status paco_verify_rows_f64(paco_ctx ctx, int64_t n, int64_t m, int64_t k,
                                 const float* A, const float* B, const float* C,
                                 const int64_t* rows, int64_t nrows, double* out);

/* --------------------------------------------------------------- timing */

/* Per-kernel timing for profiling.  While enabled, every call records HIP
 * events on the context stream around each kernel it launches.  `read`
 * synchronises the stream, sums the elapsed times by kernel role since the
 * last read (or enable) and clears them. */
typedef struct paco_timing {
  int32_t launches;     /* main-kernel launches timed */
  double main_ms;       /* semiring / ring kernels (the piece execution) */
  double reduce_ms;     /* k-cut reductions */
  double other_ms;      /* Strassen pre-add and combine, fills */
} paco_timing;

paco_status paco_timing_enable(paco_ctx ctx, int enable);
paco_status paco_timing_read(paco_ctx ctx, paco_timing* out);

/* ------------------------------------------------------------ partition */

typedef struct paco_piece {
  int64_t n0, n1, m0, m1, k0, k1;  /* half-open ranges of the cuboid */
  int32_t proc;                    /* processor it is assigned to */
  int32_t temp;                    /* 1: writes a temporary face (k0 > 0) */
  int32_t round;                   /* assignment round (multi-piece mode),
                                      0 for MM-1-Piece */
  int32_t depth;                   /* number of cuts from the root cuboid */
} paco_piece;

typedef struct paco_part_opts {
  int32_t p;                 /* processors, >= 1 */
  int32_t q_n, q_m, q_k;     /* cut quanta (cuts land on multiples); 0 = 1 */
  const double* weights;     /* NULL: equal processors; else p throughputs,
                                cuts split in the ratio of the two halves'
                                summed throughput (heterogeneous variant) */
  int32_t multi_piece;       /* 1: PACO MM pruned-BFS multi-piece mode */
  double kcut_cost;          /* see paco_mm_desc (0 = 1, the paper's rule) */
  int32_t max_rounds;        /* multi-piece: after this many rounds of p
                                pieces hand out the rest round-robin
                                (0 = divide down to the quanta) */
  int32_t tile_balance;      /* MM-1-Piece only; 1: the quanta are a kernel's
                                tile sides, and a cut that cannot land evenly
                                on them gives way to a nearly as long
                                dimension that can (how the ring product
                                plans its pieces); 0: the paper's rule */
} paco_part_opts;

/* Host-only.  Partition the n-by-m-by-k cuboid over opts->p processors.
 * Writes at most `cap` pieces to `out` and the total count to *n_out
 * (call with cap = 0 to size the array).  MM-1-Piece gives exactly p pieces
 * (possibly empty ones for tiny problems); multi-piece mode gives the
 * pruned-BFS assignment of section "PACO MM". */
paco_status paco_partition(int64_t n, int64_t m, int64_t k, const paco_part_opts* opts,
                           paco_piece* out, int64_t cap, int64_t* n_out);

/* Host-only introspection of the plan a semiring MM call launches (for
 * tests and tools; no device memory is touched).  p = 0 (PACO mode) makes
 * the default choice of a call with p = 0, using the runtime's occupancy
 * figures where a device is present and 1 workgroup per compute unit
 * otherwise.  Call once with all arrays NULL
 * to get the sizes in *info, then again with arrays of at least those sizes
 * (the counts in *info on input are the capacities):
 *   items : n_items x 8 int64 (prob, n0, n1, m0, m1, k0, k1, out_off), in
 *           kernel units (boolean m counts words); out_off < 0 writes C,
 *           otherwise a temporary face of (n1-n0) x (m1-m0) elements at
 *           that workspace offset;
 *   wg_off: n_wg + 1 int32, items of workgroup q are wg_off[q]..wg_off[q+1];
 *   tiles : n_tiles x 7 int32 (prob, i0, i1, j0, j1, s0, s1), reduction
 *           rectangles of C that fold sources s0..s1-1 in order;
 *   srcs  : n_srcs x 4 int64 (off, ld, r0, c0), element (i, j) of a source
 *           at workspace offset off + (i - r0) * ld + (j - c0).
 * num_cus is the processor count used for the grid's default split-k. */
typedef struct paco_plan_info {
  int32_t n_wg, n_items, n_tiles, n_srcs;
  int32_t tile, red_vec, xcd_remap;
  int64_t temp_elems;
  int32_t fused;                /* 1: the product kernel folds the temporary
                                   faces (each tile is one reduction cell,
                                   folded by the last piece covering it to
                                   finish); 0: a separate fold launch */
  int32_t n_fold_list;          /* fused: entries of the item -> cell lists */
} paco_plan_info;

paco_status paco_plan_export(int64_t n, int64_t m, int64_t k, paco_semiring sr, paco_part_mode part,
                             int32_t p, int32_t split_k, paco_precision prec, int32_t num_cus,
                             paco_plan_info* info, int64_t* items, int32_t* wg_off, int32_t* tiles,
                             int64_t* srcs);
/* Host-only: the fused-fold tables of the same plan (info as above): per
 * tile the number of pieces covering the cell (pads[n_tiles]); per item the
 * (begin, count) of the cells it covers in fold_list (item_fold[2 n_items],
 * fold_list[n_fold_list]).  NULL arrays fill info only. */
paco_status paco_plan_export_fold(int64_t n, int64_t m, int64_t k, paco_semiring sr, paco_part_mode part,
                                  int32_t p, int32_t split_k, paco_precision prec, int32_t num_cus,
                                  paco_plan_info* info, int32_t* pads, int32_t* item_fold, int32_t* fold_list);

#ifdef __cplusplus
}
#endif

#endif /* PACO_H */

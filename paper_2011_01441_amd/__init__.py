"""Python binding of libpaco: PACO-partitioned semiring matrix multiplication
and Strassen's algorithm on one MI355X.

Argument marshalling only: every step runs in the HIP kernels of libpaco.so.
PyTorch provides device memory and the current stream.  `torch` is imported
before the library is loaded so that libpaco binds to the HIP runtime torch
has already loaded (both carry the soname libamdhip64.so.7).
"""
import ctypes
import os

import torch

__all__ = ["Context", "Server", "PacoError", "semiring_mm", "strassen_mm", "partition", "plan_export",
           "batch_partition", "server_clock", "lib",
           "SEMIRING", "PRECISION", "INF", "NEG_INF", "library_path"]

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libpaco.so")

INF = 1 << 30
NEG_INF = -(1 << 30)
SEMIRING = {"ring": 0, "plus_times": 0, "minplus": 1, "maxplus": 2, "bool": 3}
PRECISION = {"fp32": 0, "bf16x3": 1, "bf16x6": 2, "auto": 3}
PRECISION_NAME = {v: k for k, v in PRECISION.items()}
PART = {"paco": 0, "grid": 1, "multi": 2}
_DTYPE = {0: torch.float32, 1: torch.int32, 2: torch.int32, 3: torch.int32}


class PacoError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libpaco status {status}: {msg}")
        self.status = status


class MMDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("k", ctypes.c_int64),
                ("sr", ctypes.c_int),
                ("A", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("B", ctypes.c_void_p), ("ldb", ctypes.c_int64),
                ("C", ctypes.c_void_p), ("ldc", ctypes.c_int64),
                ("accumulate", ctypes.c_int32), ("precision", ctypes.c_int),
                ("part", ctypes.c_int), ("p", ctypes.c_int32),
                ("grid_split_k", ctypes.c_int32), ("verify_rows", ctypes.c_int32),
                ("verify_seed", ctypes.c_uint64), ("kcut_cost", ctypes.c_double),
                ("weights", ctypes.c_void_p)]


class MMResult(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("p", ctypes.c_int32), ("n_pieces", ctypes.c_int32),
                ("max_piece_volume", ctypes.c_int64), ("min_piece_volume", ctypes.c_int64),
                ("temp_elems", ctypes.c_int64), ("n_kcuts", ctypes.c_int32),
                ("verify_max_rel", ctypes.c_double), ("verify_max_abs", ctypes.c_double),
                ("kcut_cost", ctypes.c_double)]


class Dp1dDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("w_kind", ctypes.c_int32), ("a", ctypes.c_int32),
                ("b", ctypes.c_int32), ("seed", ctypes.c_uint32), ("part", ctypes.c_int32),
                ("p", ctypes.c_int32), ("base", ctypes.c_int32), ("min_piece", ctypes.c_int32),
                ("D", ctypes.c_void_p)]


class Dp1dResult(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("launches", ctypes.c_int32), ("triangles", ctypes.c_int64),
                ("squares", ctypes.c_int64), ("pieces", ctypes.c_int64), ("max_pieces", ctypes.c_int32),
                ("atomic_pieces", ctypes.c_int32)]


W_KIND = {"affine": 0, "hash": 1}


class Weight(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("a", ctypes.c_int32), ("b", ctypes.c_int32), ("seed", ctypes.c_uint32)]


class GapDesc(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("w_row", Weight), ("w_col", Weight),
                ("s_match", ctypes.c_int32), ("s_mismatch", ctypes.c_int32), ("s_bits", ctypes.c_int32),
                ("s_seed_x", ctypes.c_uint32), ("s_seed_y", ctypes.c_uint32), ("part", ctypes.c_int32),
                ("p", ctypes.c_int32), ("min_piece", ctypes.c_int32), ("D", ctypes.c_void_p),
                ("ldd", ctypes.c_int64)]


class GapResult(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("launches", ctypes.c_int32), ("base_blocks", ctypes.c_int64),
                ("cubes", ctypes.c_int64), ("pieces", ctypes.c_int64)]


def _weight(w):
    """(kind, a, b, seed) -> Weight"""
    return Weight(W_KIND[w[0]], w[1], w[2], w[3] & 0xFFFFFFFF)


class StrassenDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("A", ctypes.c_void_p), ("B", ctypes.c_void_p), ("C", ctypes.c_void_p),
                ("p", ctypes.c_int32), ("gamma", ctypes.c_int32), ("base", ctypes.c_int64),
                ("leaf", ctypes.c_int)]


class StrassenResult(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("super_rounds", ctypes.c_int32), ("max_depth", ctypes.c_int32),
                ("nodes", ctypes.c_int64), ("max_work", ctypes.c_double), ("min_work", ctypes.c_double),
                ("temp_bytes", ctypes.c_uint64), ("leaf", ctypes.c_int)]


class TuneResult(ctypes.Structure):
    _fields_ = [("tuned", ctypes.c_int32), ("part", ctypes.c_int), ("p", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("weighted", ctypes.c_int32), ("kcut_cost", ctypes.c_double),
                ("best_ms", ctypes.c_double), ("default_ms", ctypes.c_double),
                ("candidates", ctypes.c_int32)]


class StrassenLevel(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("super_round", ctypes.c_int32), ("h", ctypes.c_int64),
                ("nodes", ctypes.c_int64), ("assigned", ctypes.c_int64)]


class Piece(ctypes.Structure):
    _fields_ = [("n0", ctypes.c_int64), ("n1", ctypes.c_int64), ("m0", ctypes.c_int64),
                ("m1", ctypes.c_int64), ("k0", ctypes.c_int64), ("k1", ctypes.c_int64),
                ("proc", ctypes.c_int32), ("temp", ctypes.c_int32),
                ("round", ctypes.c_int32), ("depth", ctypes.c_int32)]


class Timing(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int32), ("main_ms", ctypes.c_double),
                ("reduce_ms", ctypes.c_double), ("other_ms", ctypes.c_double)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_wg", ctypes.c_int32), ("n_items", ctypes.c_int32), ("n_tiles", ctypes.c_int32),
                ("n_srcs", ctypes.c_int32), ("tile", ctypes.c_int32), ("red_vec", ctypes.c_int32),
                ("xcd_remap", ctypes.c_int32), ("temp_elems", ctypes.c_int64), ("fused", ctypes.c_int32),
                ("n_fold_list", ctypes.c_int32)]


class PartOpts(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("q_n", ctypes.c_int32), ("q_m", ctypes.c_int32),
                ("q_k", ctypes.c_int32), ("weights", ctypes.POINTER(ctypes.c_double)),
                ("multi_piece", ctypes.c_int32), ("kcut_cost", ctypes.c_double),
                ("max_rounds", ctypes.c_int32), ("tile_balance", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("k", ctypes.c_int64),
                ("sr", ctypes.c_int),
                ("A", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("B", ctypes.c_void_p), ("ldb", ctypes.c_int64),
                ("C", ctypes.c_void_p), ("ldc", ctypes.c_int64),
                ("precision", ctypes.c_int), ("arrival_s", ctypes.c_double)]


class RequestResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("precision", ctypes.c_int),
                ("arrival_s", ctypes.c_double), ("launch_s", ctypes.c_double),
                ("done_s", ctypes.c_double), ("batch_id", ctypes.c_int32),
                ("batch_size", ctypes.c_int32)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_batch", ctypes.c_int32),
                ("per_request", ctypes.c_int32), ("p", ctypes.c_int32),
                ("batch_window_s", ctypes.c_double), ("spin_s", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("mean_batch", ctypes.c_double), ("p50_s", ctypes.c_double),
                ("p99_s", ctypes.c_double), ("max_s", ctypes.c_double),
                ("span_s", ctypes.c_double), ("ops", ctypes.c_double),
                ("retained", ctypes.c_int64), ("bytes_in_flight", ctypes.c_uint64)]


_lib = None


def lib():
    """Load libpaco.so; raises if it has not been built (no CPU fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(library_path):
        raise ImportError(f"{library_path} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(library_path)
    vp, i64, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    L.paco_create.argtypes = [ctypes.POINTER(vp), ci, ctypes.c_uint64]
    L.paco_destroy.argtypes = [vp]
    L.paco_set_stream.argtypes = [vp, vp]
    L.paco_num_cus.argtypes = [vp]
    L.paco_set_piece_stamps.argtypes = [vp, vp, ctypes.c_int32]
    L.paco_set_piece_stamps.restype = ci
    L.paco_num_cus.restype = ci
    L.paco_status_string.argtypes = [ci]
    L.paco_status_string.restype = ctypes.c_char_p
    L.paco_last_error.argtypes = [vp]
    L.paco_last_error.restype = ctypes.c_char_p
    L.paco_semiring_mm.argtypes = [vp, i64, i64, i64, ci, vp, vp, vp]
    L.paco_semiring_mm_ex.argtypes = [vp, ctypes.POINTER(MMDesc), ctypes.POINTER(MMResult)]
    L.paco_mm_validate.argtypes = [ctypes.POINTER(MMDesc)]
    L.paco_semiring_mm_noalloc.argtypes = [vp, ctypes.POINTER(MMDesc), ctypes.POINTER(MMResult)]
    L.paco_noalloc_scratch_bytes.argtypes = []
    L.paco_noalloc_scratch_bytes.restype = ctypes.c_uint64
    L.paco_strassen_mm.argtypes = [vp, i64, vp, vp, vp, ci, ci]
    L.paco_calibrate.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp]
    L.paco_tune.argtypes = [vp, ctypes.POINTER(MMDesc), ctypes.POINTER(TuneResult)]
    L.paco_tune_clear.argtypes = [vp]
    L.paco_graph_create.argtypes = [vp, ctypes.POINTER(MMDesc), ctypes.c_int32, ctypes.POINTER(vp)]
    L.paco_graph_create_strassen.argtypes = [vp, ctypes.POINTER(StrassenDesc), ctypes.c_int32,
                                             ctypes.POINTER(vp)]
    L.paco_graph_launch.argtypes = [vp, vp]
    L.paco_graph_destroy.argtypes = [vp]
    L.paco_set_processor_weights.argtypes = [vp, ctypes.c_int32, vp]
    L.paco_peak.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    L.paco_strassen_pbfs.argtypes = [vp, ctypes.POINTER(StrassenDesc), ctypes.POINTER(StrassenResult)]
    L.paco_dp1d.argtypes = [vp, ctypes.POINTER(Dp1dDesc), ctypes.POINTER(Dp1dResult)]
    L.paco_gap.argtypes = [vp, ctypes.POINTER(GapDesc), ctypes.POINTER(GapResult)]
    L.paco_gap_plan_export.argtypes = [i64, i64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp]
    L.paco_dp1d_plan_export.argtypes = [i64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                        vp, vp, vp]
    L.paco_strassen_schedule.argtypes = [i64, ctypes.c_int32, ctypes.c_int32, i64,
                                         ctypes.POINTER(StrassenLevel), ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int32), vp, vp]
    L.paco_verify_rows_f64.argtypes = [vp, i64, i64, i64, vp, vp, vp, vp, i64,
                                       ctypes.POINTER(ctypes.c_double)]
    L.paco_partition.argtypes = [i64, i64, i64, ctypes.POINTER(PartOpts), ctypes.POINTER(Piece),
                                 i64, ctypes.POINTER(i64)]
    L.paco_plan_export.argtypes = [i64, i64, i64, ci, ci, ctypes.c_int32, ctypes.c_int32, ci,
                                   ctypes.c_int32, ctypes.POINTER(PlanInfo), vp, vp, vp, vp]
    L.paco_plan_export_fold.argtypes = [i64, i64, i64, ci, ci, ctypes.c_int32, ctypes.c_int32, ci,
                                        ctypes.c_int32, ctypes.POINTER(PlanInfo), vp, vp, vp]
    L.paco_plan_export_fold.restype = ci
    L.paco_server_clock.restype = ctypes.c_double
    L.paco_server_create.argtypes = [vp, ctypes.POINTER(ServerOpts), ctypes.POINTER(vp)]
    L.paco_server_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    L.paco_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ci), ctypes.POINTER(RequestResult)]
    L.paco_server_drain.argtypes = [vp]
    L.paco_server_stats_get.argtypes = [vp, ctypes.POINTER(ServerStats)]
    L.paco_server_destroy.argtypes = [vp]
    L.paco_server_fail_batches.argtypes = [vp, ctypes.c_int32]
    L.paco_batch_partition.argtypes = [ctypes.POINTER(Request), ctypes.c_int32, ctypes.c_int32,
                                       ctypes.POINTER(Piece), ctypes.POINTER(ctypes.c_int32), i64,
                                       ctypes.POINTER(i64)]
    L.paco_timing_enable.argtypes = [vp, ci]
    L.paco_timing_read.argtypes = [vp, ctypes.POINTER(Timing)]
    for name in ("paco_server_create", "paco_server_submit", "paco_server_poll",
                 "paco_server_drain", "paco_server_stats_get", "paco_server_destroy", "paco_server_fail_batches",
                 "paco_batch_partition", "paco_plan_export", "paco_timing_enable", "paco_timing_read", "paco_create", "paco_destroy", "paco_set_stream", "paco_semiring_mm",
                 "paco_semiring_mm_ex", "paco_semiring_mm_noalloc", "paco_mm_validate", "paco_strassen_mm", "paco_verify_rows_f64",
                 "paco_partition"):
        getattr(L, name).restype = ci
    _lib = L
    return L


def _check(st, ctx=None):
    if st != 0:
        L = lib()
        msg = L.paco_last_error(ctx).decode() if ctx else ""
        raise PacoError(st, f"{L.paco_status_string(st).decode()}: {msg}")


def strassen_schedule(n, p, gamma=0, base=256):
    """Host-only: the pruned-BFS schedule of PACO Strassen.  Returns (levels,
    work_classic, work_strassen): one dict per depth (depth, super_round, h,
    nodes, assigned) and per-processor sums of h^3 and h^log2(7)."""
    import numpy as np
    L = lib()
    nl = ctypes.c_int32()
    _check(L.paco_strassen_schedule(n, p, gamma, base, None, 0, ctypes.byref(nl), None, None))
    lv = (StrassenLevel * max(nl.value, 1))()
    wc = np.zeros(p, np.float64)
    wsr = np.zeros(p, np.float64)
    _check(L.paco_strassen_schedule(n, p, gamma, base, lv, nl.value, ctypes.byref(nl),
                                    ctypes.c_void_p(wc.ctypes.data), ctypes.c_void_p(wsr.ctypes.data)))
    levels = [{f[0]: getattr(lv[i], f[0]) for f in StrassenLevel._fields_} for i in range(nl.value)]
    return levels, wc, wsr


def dp1d_plan(n, part="paco", p=1024, base=512, min_piece=65536):
    """Host-only: the plan of paco_dp1d.  Returns (first_len, triangles,
    squares, pieces): squares an (S, 8) int64 array (lo, mid, hi, first
    piece, piece count, tri_lo, tri_len, pieces reaching the triangle),
    pieces a (P, 5) int64 array (i0, i1, j0, j1, inputs cut)."""
    import numpy as np
    L = lib()
    info = np.zeros(4, np.int64)
    vp = lambda a: ctypes.c_void_p(a.ctypes.data)
    _check(L.paco_dp1d_plan_export(n, PART[part], p, base, min_piece, vp(info), None, None))
    sq = np.zeros((max(int(info[0]), 1), 8), np.int64)
    pc = np.zeros((max(int(info[1]), 1), 5), np.int64)
    _check(L.paco_dp1d_plan_export(n, PART[part], p, base, min_piece, vp(info), vp(sq), vp(pc)))
    return int(info[2]), int(info[3]), sq[:int(info[0])], pc[:int(info[1])]


def gap_plan(m, n, part="paco", p=1024, min_piece=65536):
    """Host-only: the plan of paco_gap.  Returns (launches, blocks, pieces,
    cubes): launches an (L, 3) int64 array (1 base / 0 cubes, first entry,
    count), blocks (B, 4) (r0, r1, c0, c1), pieces (P, 7) (column-gap flag,
    t0, t1, x0, x1, o0, o1)."""
    import numpy as np
    L = lib()
    info = np.zeros(4, np.int64)
    vp = lambda a: ctypes.c_void_p(a.ctypes.data)
    _check(L.paco_gap_plan_export(m, n, PART[part], p, min_piece, vp(info), None, None, None))
    la = np.zeros((max(int(info[0]), 1), 3), np.int64)
    bl = np.zeros((max(int(info[1]), 1), 4), np.int64)
    pc = np.zeros((max(int(info[2]), 1), 7), np.int64)
    _check(L.paco_gap_plan_export(m, n, PART[part], p, min_piece, vp(info), vp(la), vp(bl), vp(pc)))
    return la[:int(info[0])], bl[:int(info[1])], pc[:int(info[2])], int(info[3])


def partition(n, m, k, p, q=(1, 1, 1), weights=None, multi_piece=False, kcut_cost=1.0, max_rounds=0,
              tile_balance=False):
    """Host-only PACO partition (MM-1-Piece, or pruned-BFS multi-piece):
    a list of dicts with n0,n1,m0,m1,k0,k1, proc, temp, round, depth."""
    L = lib()
    o = PartOpts(p, q[0], q[1], q[2], None, 1 if multi_piece else 0, kcut_cost, max_rounds,
                 1 if tile_balance else 0)
    if weights is not None:
        arr = (ctypes.c_double * p)(*[float(w) for w in weights])
        o.weights = ctypes.cast(arr, ctypes.POINTER(ctypes.c_double))
    cnt = ctypes.c_int64(0)
    _check(L.paco_partition(n, m, k, ctypes.byref(o), None, 0, ctypes.byref(cnt)))
    buf = (Piece * max(cnt.value, 1))()
    _check(L.paco_partition(n, m, k, ctypes.byref(o), buf, cnt.value, ctypes.byref(cnt)))
    names = [f[0] for f in Piece._fields_]
    return [{f: getattr(buf[i], f) for f in names} for i in range(cnt.value)]


def plan_export(n, m, k, semiring, part="paco", p=256, split_k=0, precision="auto",
                num_cus=256):
    """Host-only: the work plan of a semiring MM call, as numpy arrays
    (items n x 8, wg_off, tiles n x 7, srcs n x 4) plus an info dict."""
    import numpy as np
    L = lib()
    info = PlanInfo()
    args = (n, m, k, SEMIRING[semiring], PART[part], p, split_k, PRECISION[precision], num_cus)
    _check(L.paco_plan_export(*args, ctypes.byref(info), None, None, None, None))
    items = np.zeros((max(info.n_items, 1), 8), np.int64)
    wg = np.zeros(info.n_wg + 1, np.int32)
    tiles = np.zeros((max(info.n_tiles, 1), 7), np.int32)
    srcs = np.zeros((max(info.n_srcs, 1), 4), np.int64)
    ptr = lambda a: ctypes.c_void_p(a.ctypes.data)
    _check(L.paco_plan_export(*args, ctypes.byref(info), ptr(items), ptr(wg), ptr(tiles), ptr(srcs)))
    d = {f[0]: getattr(info, f[0]) for f in PlanInfo._fields_}
    return (items[:info.n_items], wg, tiles[:info.n_tiles], srcs[:info.n_srcs], d)


def plan_export_fold(n, m, k, semiring, part="paco", p=256, split_k=0, precision="auto", num_cus=256):
    """Host-only: the fused-fold tables of the plan plan_export returns:
    (pads per tile, item_fold (n_items x 2), fold_list, info)."""
    import numpy as np
    L = lib()
    info = PlanInfo()
    args = (n, m, k, SEMIRING[semiring], PART[part], p, split_k, PRECISION[precision], num_cus)
    _check(L.paco_plan_export_fold(*args, ctypes.byref(info), None, None, None))
    pads = np.zeros(max(info.n_tiles, 1), np.int32)
    itf = np.zeros((max(info.n_items, 1), 2), np.int32)
    fl = np.zeros(max(info.n_fold_list, 1), np.int32)
    ptr = lambda a: ctypes.c_void_p(a.ctypes.data)
    _check(L.paco_plan_export_fold(*args, ctypes.byref(info), ptr(pads), ptr(itf), ptr(fl)))
    d = {f[0]: getattr(info, f[0]) for f in PlanInfo._fields_}
    return pads[:info.n_tiles], itf[:info.n_items], fl[:info.n_fold_list], d


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


class Graph:
    """A captured library call (paco_graph); launch() replays it on torch's
    current stream.  Keeps its operand tensors alive."""

    def __init__(self, ctx, h, keep):
        self._ctx, self._h, self._keep = ctx, h, keep

    def launch(self):
        s = torch.cuda.current_stream(self._ctx.device).cuda_stream
        _check(self._ctx._L.paco_graph_launch(self._h, ctypes.c_void_p(s)), self._ctx._h)

    def close(self):
        if self._h:
            self._ctx._L.paco_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """A libpaco context on one device; launches on torch's current stream."""

    def __init__(self, device=0, workspace_budget=0):
        self._L = lib()
        self.device = device
        h = ctypes.c_void_p()
        _check(self._L.paco_create(ctypes.byref(h), device, workspace_budget))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._L.paco_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_piece_stamps(self, stamps=None):
        """stamps: an int64 device tensor of shape (P, 4), or None.  Later
        semiring MM calls record, per processor q < P: start and end of its
        work (100 MHz device clock), XCC_ID and HW_ID registers."""
        if stamps is None:
            _check(self._L.paco_set_piece_stamps(self._h, None, 0), self._h)
            self._stamps = None
            return
        if (stamps.dtype != torch.int64 or stamps.dim() != 2 or stamps.shape[1] != 4 or not stamps.is_contiguous()
                or stamps.device.type != "cuda"):
            raise ValueError("stamps must be a contiguous int64 (P, 4) device tensor")
        _check(self._L.paco_set_piece_stamps(self._h, _ptr(stamps), stamps.shape[0]), self._h)
        self._stamps = stamps   # kept alive while set

    @property
    def num_cus(self):
        return self._L.paco_num_cus(self._h)

    def _stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        _check(self._L.paco_set_stream(self._h, ctypes.c_void_p(s)), self._h)

    def _check_tensor(self, t, name, dtype):
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.device.index != self.device:
            raise ValueError(f"{name} must be a tensor on cuda:{self.device}")
        if t.dtype != dtype:
            raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
        if t.dim() != 2 or t.stride(1) != 1:
            raise ValueError(f"{name} must be 2-D with unit column stride")

    def tune(self, A, B, semiring="ring", **kw):
        """Time the default plan of this shape and its alternatives on these
        operands (C is overwritten); keep the fastest for later default
        calls.  Returns the tuner's result as a dict."""
        if kw.get("C") is None:
            raise ValueError("tuning needs the output buffer C")
        d, keep = self._desc(A, B, semiring, **kw)
        r = TuneResult()
        self._stream()
        _check(self._L.paco_tune(self._h, ctypes.byref(d), ctypes.byref(r)), self._h)
        out = {f[0]: getattr(r, f[0]) for f in TuneResult._fields_}
        out["part"] = {v: k for k, v in PART.items()}.get(out["part"], out["part"])
        return out

    def tune_clear(self):
        _check(self._L.paco_tune_clear(self._h), self._h)

    def graph(self, A, B, semiring="ring", repeat=1, **kw):
        """Capture `repeat` runs of C = A (x) B (same arguments as
        semiring_mm, C required) into a hipGraph; returns a Graph whose
        launch() replays them."""
        if kw.get("C") is None:
            raise ValueError("a captured call needs its output buffer C")
        d, keep = self._desc(A, B, semiring, **kw)
        self._stream()
        h = ctypes.c_void_p()
        _check(self._L.paco_graph_create(self._h, ctypes.byref(d), repeat, ctypes.byref(h)), self._h)
        return Graph(self, h, (A, B, kw["C"], keep))

    def graph_strassen(self, A, B, C, p=0, gamma=0, base=0, leaf="bf16x3", repeat=1):
        """Capture a pruned-BFS Strassen call into a hipGraph."""
        for t, nm in ((A, "A"), (B, "B"), (C, "C")):
            self._check_tensor(t, nm, torch.float32)
        n = A.shape[0]
        if A.shape != (n, n) or B.shape != (n, n) or C.shape != (n, n) or not all(
                t.is_contiguous() for t in (A, B, C)):
            raise ValueError("Strassen needs dense square operands of equal size")
        d = StrassenDesc(n, _ptr(A), _ptr(B), _ptr(C), p, gamma, base, PRECISION[leaf])
        self._stream()
        h = ctypes.c_void_p()
        _check(self._L.paco_graph_create_strassen(self._h, ctypes.byref(d), repeat, ctypes.byref(h)), self._h)
        return Graph(self, h, (A, B, C))

    def _desc(self, A, B, semiring="ring", *, n=None, m=None, k=None, C=None, accumulate=False,
              precision="auto", part="paco", p=0, split_k=0, verify_rows=0, verify_seed=0, kcut_cost=0.0,
              weights=None):
        sr = SEMIRING[semiring]
        dt = _DTYPE[sr]
        self._check_tensor(A, "A", dt)
        self._check_tensor(B, "B", dt)
        if sr == 3:
            if n is None or m is None or k is None:
                raise ValueError("boolean operands need explicit n, m, k (bits)")
        else:
            n, k = A.shape
            k2, m = B.shape
            if k2 != k:
                raise ValueError(f"inner sizes differ: {A.shape} x {B.shape}")
        self._check_tensor(C, "C", dt)
        w = None
        if weights is not None:
            import numpy as np
            w = np.ascontiguousarray(weights, np.float64)
            if w.shape != (p,):
                raise ValueError("weights need one entry per processor (explicit p)")
        d = MMDesc(n, m, k, sr, _ptr(A), A.stride(0), _ptr(B), B.stride(0), _ptr(C), C.stride(0),
                   1 if accumulate else 0, PRECISION[precision], PART[part], p, split_k,
                   verify_rows, verify_seed, kcut_cost,
                   ctypes.c_void_p(w.ctypes.data) if w is not None else None)
        return d, w

    def semiring_mm(self, A, B, semiring="ring", **kw):
        """C = A (x) B.  Boolean operands are bit-packed int32 words; pass
        their logical sizes n, m, k.  Returns C (and a result dict)."""
        return self._mm(self._L.paco_semiring_mm_ex, A, B, semiring, **kw)

    def semiring_mm_noalloc(self, A, B, semiring="ring", **kw):
        """As semiring_mm, through the entry point that allocates no device
        memory (paco_semiring_mm_noalloc): C must be given."""
        if kw.get("C") is None:
            raise ValueError("the allocation-free call needs its output buffer C")
        return self._mm(self._L.paco_semiring_mm_noalloc, A, B, semiring, **kw)

    def _mm(self, fn, A, B, semiring="ring", *, n=None, m=None, k=None, C=None,
            accumulate=False, precision="auto", part="paco", p=0, split_k=0,
            verify_rows=0, verify_seed=0, kcut_cost=0.0, weights=None, return_result=False):
        sr = SEMIRING[semiring]
        dt = _DTYPE[sr]
        self._check_tensor(A, "A", dt)
        self._check_tensor(B, "B", dt)
        if sr == 3:
            if n is None or m is None or k is None:
                raise ValueError("boolean operands need explicit n, m, k (bits)")
            mw = (m + 31) // 32
        else:
            n, k = A.shape
            k2, m = B.shape
            if k2 != k:
                raise ValueError(f"inner sizes differ: {A.shape} x {B.shape}")
            mw = m
        if C is None:
            C = torch.empty((n, mw), dtype=dt, device=A.device)
        else:
            self._check_tensor(C, "C", dt)
        w = None
        if weights is not None:
            import numpy as np
            w = np.ascontiguousarray(weights, np.float64)
            if w.shape != (p,):
                raise ValueError("weights need one entry per processor (explicit p)")
        d = MMDesc(n, m, k, sr, _ptr(A), A.stride(0), _ptr(B), B.stride(0), _ptr(C), C.stride(0),
                   1 if accumulate else 0, PRECISION[precision], PART[part], p, split_k,
                   verify_rows, verify_seed, kcut_cost,
                   ctypes.c_void_p(w.ctypes.data) if w is not None else None)
        r = MMResult()
        self._stream()
        _check(fn(self._h, ctypes.byref(d), ctypes.byref(r)), self._h)
        if not return_result:
            return C
        res = {f[0]: getattr(r, f[0]) for f in MMResult._fields_}
        res["precision"] = PRECISION_NAME.get(res["precision"], res["precision"])
        return C, res

    def strassen_mm(self, A, B, levels=2, leaf="bf16x3", C=None):
        self._check_tensor(A, "A", torch.float32)
        self._check_tensor(B, "B", torch.float32)
        n = A.shape[0]
        if A.shape != (n, n) or B.shape != (n, n) or not A.is_contiguous() or not B.is_contiguous():
            raise ValueError("Strassen needs dense square operands of equal size")
        if C is None:
            C = torch.empty((n, n), dtype=torch.float32, device=A.device)
        self._stream()
        _check(self._L.paco_strassen_mm(self._h, n, _ptr(A), _ptr(B), _ptr(C), levels,
                                        PRECISION[leaf]), self._h)
        return C

    def calibrate(self, p=0, iters=0):
        """Measured throughput (bf16 TFLOP/s) of each of p processors
        (default: compute units), for semiring_mm(weights=...)."""
        import numpy as np
        p = p or self._L.paco_num_cus(self._h)
        r = np.zeros(p, np.float64)
        self._stream()
        _check(self._L.paco_calibrate(self._h, p, iters, ctypes.c_void_p(r.ctypes.data)), self._h)
        return r

    def peak(self, kind):
        """Measured peak of this device: "mfma_bf16" (TFLOP/s), "valu_i32"
        (T lane-instructions/s of u32 add and min), "valu_f32" (TFLOP/s of
        unpacked FMA) or "hbm_copy" (GB/s read + written)."""
        kinds = {"mfma_bf16": 0, "valu_i32": 1, "valu_f32": 2, "hbm_copy": 3}
        r = ctypes.c_double(0.0)
        self._stream()
        _check(self._L.paco_peak(self._h, kinds[kind], ctypes.byref(r)), self._h)
        return r.value

    def set_processor_weights(self, weights=None):
        """Default-p ring calls in PACO mode use these throughputs (one per
        compute unit); None clears them."""
        import numpy as np
        if weights is None:
            _check(self._L.paco_set_processor_weights(self._h, 0, None), self._h)
            return
        w = np.ascontiguousarray(weights, np.float64)
        _check(self._L.paco_set_processor_weights(self._h, len(w), ctypes.c_void_p(w.ctypes.data)), self._h)

    def dp1d(self, D, kind, a, b, seed=0, part="paco", p=0, base=0, min_piece=0, return_result=False):
        """The 1D problem (section "PACO 1D") in place on D, an int32 tensor
        of n + 1 entries: D[0] is read, D[1..n] are written."""
        if not isinstance(D, torch.Tensor) or D.device.type != "cuda" or D.device.index != self.device:
            raise ValueError(f"D must be a tensor on cuda:{self.device}")
        if D.dtype != torch.int32 or D.dim() != 1 or not D.is_contiguous() or D.numel() < 1:
            raise ValueError("D must be a contiguous 1-D int32 tensor of n + 1 entries")
        d = Dp1dDesc(D.numel() - 1, W_KIND[kind], a, b, seed & 0xFFFFFFFF, PART[part], p, base, min_piece,
                     _ptr(D))
        r = Dp1dResult()
        self._stream()
        _check(self._L.paco_dp1d(self._h, ctypes.byref(d), ctypes.byref(r)), self._h)
        if return_result:
            return D, {f[0]: getattr(r, f[0]) for f in Dp1dResult._fields_}
        return D

    def gap(self, D, w_row, w_col, s, part="paco", p=0, min_piece=0, return_result=False):
        """The GAP problem (section "PACO GAP") in place on D, an (m+1) x (n+1)
        int32 tensor (unit column stride): D[0, 0] is read, every cell is
        written.  w_row, w_col: (kind, a, b, seed); s: (s_match, s_mismatch,
        bits, seed_x, seed_y)."""
        if not isinstance(D, torch.Tensor) or D.device.type != "cuda" or D.device.index != self.device:
            raise ValueError(f"D must be a tensor on cuda:{self.device}")
        if D.dtype != torch.int32 or D.dim() != 2 or D.stride(1) != 1 or D.shape[0] < 1 or D.shape[1] < 1:
            raise ValueError("D must be a 2-D int32 tensor with unit column stride")
        d = GapDesc(D.shape[0] - 1, D.shape[1] - 1, _weight(w_row), _weight(w_col), s[0], s[1], s[2],
                    s[3] & 0xFFFFFFFF, s[4] & 0xFFFFFFFF, PART[part], p, min_piece, _ptr(D), D.stride(0))
        r = GapResult()
        self._stream()
        _check(self._L.paco_gap(self._h, ctypes.byref(d), ctypes.byref(r)), self._h)
        if return_result:
            return D, {f[0]: getattr(r, f[0]) for f in GapResult._fields_}
        return D

    def strassen_pbfs(self, A, B, C=None, p=0, gamma=0, base=0, leaf="bf16x3", return_result=False):
        """PACO Strassen with the pruned-BFS schedule over p processor groups
        (0: one per XCD); gamma caps the super-rounds (0: none)."""
        self._check_tensor(A, "A", torch.float32)
        self._check_tensor(B, "B", torch.float32)
        n = A.shape[0]
        if A.shape != (n, n) or B.shape != (n, n) or not A.is_contiguous() or not B.is_contiguous():
            raise ValueError("Strassen needs dense square operands of equal size")
        if C is None:
            C = torch.empty((n, n), dtype=torch.float32, device=A.device)
        elif C.shape != (n, n) or not C.is_contiguous():
            raise ValueError("C must be a dense n x n tensor")
        d = StrassenDesc(n, _ptr(A), _ptr(B), _ptr(C), p, gamma, base, PRECISION[leaf])
        r = StrassenResult()
        self._stream()
        _check(self._L.paco_strassen_pbfs(self._h, ctypes.byref(d), ctypes.byref(r)), self._h)
        if not return_result:
            return C
        res = {f[0]: getattr(r, f[0]) for f in StrassenResult._fields_}
        res["leaf"] = PRECISION_NAME.get(res["leaf"], res["leaf"])
        return C, res

    def timing(self, enable=None):
        """timing(True) starts per-kernel event timing; timing() reads and
        clears it: dict(launches, main_ms, reduce_ms, other_ms)."""
        if enable is not None:
            _check(self._L.paco_timing_enable(self._h, 1 if enable else 0), self._h)
            return None
        t = Timing()
        _check(self._L.paco_timing_read(self._h, ctypes.byref(t)), self._h)
        return {f[0]: getattr(t, f[0]) for f in Timing._fields_}

    def verify_rows(self, A, B, C, rows):
        """float64 check of the listed rows: (max rel, max abs, sum sq diff, sum sq ref)."""
        n, k = A.shape
        m = B.shape[1]
        rows = rows.to(device=A.device, dtype=torch.int64).contiguous()
        out = (ctypes.c_double * 4)()
        self._stream()
        _check(self._L.paco_verify_rows_f64(self._h, n, m, k, _ptr(A), _ptr(B), _ptr(C),
                                            _ptr(rows), rows.numel(), out), self._h)
        return tuple(out)


_default = None


def _ctx():
    global _default
    if _default is None:
        _default = Context(torch.cuda.current_device())
    return _default


def semiring_mm(A, B, semiring="ring", **kw):
    return _ctx().semiring_mm(A, B, semiring, **kw)


def strassen_mm(A, B, levels=2, leaf="bf16x3"):
    return _ctx().strassen_mm(A, B, levels, leaf)


# ------------------------------------------------------------------ server

def server_clock():
    """The monotonic clock (seconds) the server stamps request times with."""
    return lib().paco_server_clock()


def _request(n, m, k, semiring, A=0, lda=0, B=0, ldb=0, C=0, ldc=0, precision="auto", arrival=0.0):
    return Request(n, m, k, SEMIRING[semiring], A, lda, B, ldb, C, ldc, PRECISION[precision], arrival)


def batch_partition(reqs, p):
    """Host-only: pieces the server launches for a batch.  reqs: dicts with
    n, m, k, semiring (and optional precision).  Returns piece dicts with the
    request index under 'req'."""
    L = lib()
    arr = (Request * max(len(reqs), 1))(*[_request(r["n"], r["m"], r["k"], r["semiring"],
                                                   precision=r.get("precision", "auto"))
                                          for r in reqs])
    cnt = ctypes.c_int64(0)
    _check(L.paco_batch_partition(arr, len(reqs), p, None, None, 0, ctypes.byref(cnt)))
    buf = (Piece * max(cnt.value, 1))()
    rq = (ctypes.c_int32 * max(cnt.value, 1))()
    _check(L.paco_batch_partition(arr, len(reqs), p, buf, rq, cnt.value, ctypes.byref(cnt)))
    names = [f[0] for f in Piece._fields_]
    out = []
    for i in range(cnt.value):
        d = {f: getattr(buf[i], f) for f in names}
        d["req"] = rq[i]
        out.append(d)
    return out


class Server:
    """Batching request server on a device (see include/paco_server.h)."""

    def __init__(self, ctx, hbm_budget=0, max_batch=0, per_request=False, p=0, window_s=0.0, spin_s=0.0):
        self._L = lib()
        o = ServerOpts(hbm_budget, max_batch, 1 if per_request else 0, p, window_s, spin_s)
        h = ctypes.c_void_p()
        _check(self._L.paco_server_create(ctx._h, ctypes.byref(o), ctypes.byref(h)))
        self._h = h

    def submit(self, A, B, C, semiring="ring", *, n=None, m=None, k=None, precision="auto",
               arrival=0.0):
        """Queue C = A (x) B.  Tensors may be row-strided views; boolean
        operands need explicit n, m, k (bits).  Returns a ticket."""
        sr = SEMIRING[semiring]
        if sr != 3:
            n, k = A.shape
            m = B.shape[1]
        r = Request(n, m, k, sr, _ptr(A), A.stride(0), _ptr(B), B.stride(0), _ptr(C), C.stride(0),
                    PRECISION[precision], arrival)
        t = ctypes.c_uint64(0)
        _check(self._L.paco_server_submit(self._h, ctypes.byref(r), ctypes.byref(t)))
        return t.value

    def poll(self, ticket):
        done = ctypes.c_int(0)
        r = RequestResult()
        _check(self._L.paco_server_poll(self._h, ticket, ctypes.byref(done), ctypes.byref(r)))
        d = {f[0]: getattr(r, f[0]) for f in RequestResult._fields_}
        d["precision"] = PRECISION_NAME.get(d["precision"], d["precision"])
        return bool(done.value), d

    def drain(self):
        _check(self._L.paco_server_drain(self._h))

    def fail_batches(self, count):
        """Testing hook: the next `count` batches fail before launch."""
        _check(self._L.paco_server_fail_batches(self._h, count))

    def stats(self):
        st = ServerStats()
        _check(self._L.paco_server_stats_get(self._h, ctypes.byref(st)))
        return {f[0]: getattr(st, f[0]) for f in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            self._L.paco_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

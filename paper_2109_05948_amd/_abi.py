"""ctypes binding of libdlmcol.so: argument marshalling only.

Every call maps one-to-one onto a ``dlm_*`` entry point of
``include/dlmcol.h``.  torch is used for device memory (tensors' data
pointers) and streams (``torch.cuda.current_stream().cuda_stream``); every
step of the search runs in the library's HIP kernels.  There is no fallback:
if the library is missing or a call fails, a Python exception is raised.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdlmcol.so")
_lock = threading.Lock()
_lib = None

NSTATS = 8
DLM_OK = 0
TABLES = {"auto": 0, "lds16": 1, "lds32": 2, "global16": 3, "split16": 4, "split8": 5, "wave8": 6}
INIT_MODES = {"random": 0, "greedy": 1}

EXPORTS = [
    "dlm_abi_version", "dlm_last_error", "dlm_graph_create", "dlm_graph_destroy", "dlm_graph_info",
    "dlm_init_population", "dlm_tabu_workspace_bytes", "dlm_tabu_batch", "dlm_tabu_batch_static",
    "dlm_evaluate", "dlm_gpx_batch", "dlm_select",
    "dlm_wvcp_batch", "dlm_scorer_create", "dlm_scorer_destroy", "dlm_scorer_num_params",
    "dlm_scorer_get_params", "dlm_score_offspring", "dlm_scorer_grad", "dlm_scorer_train",
    "dlm_gather_rows", "dlm_standardize", "dlm_random_pairs", "dlm_pop_update",
    "dlm_multi_plan_create", "dlm_multi_plan_launch", "dlm_multi_plan_info",
    "dlm_multi_plan_destroy", "dlm_multi_autotune", "dlm_probe_lds_bandwidth",
    "dlm_partition_distance", "dlm_spacing_update", "dlm_gather_distances", "dlm_gather_pool",
    "dlm_nearest", "dlm_select_groups", "dlm_reduce_colours", "dlm_invnet_create",
    "dlm_invnet_destroy", "dlm_invnet_num_params", "dlm_invnet_get_params", "dlm_invnet_forward",
    "dlm_invnet_grad", "dlm_invnet_train", "dlm_gemm_bf16", "dlm_wvcp_targets",
]


class DlmError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} returned {code}: {msg}")
        self.code = code


class TabuParams(C.Structure):
    _fields_ = [("k", C.c_int32), ("max_iters", C.c_int32), ("ten_num", C.c_int32),
                ("ten_den", C.c_int32), ("ten_rand", C.c_int32), ("ind_base", C.c_int32),
                ("seed", C.c_uint64), ("block", C.c_int32), ("table", C.c_int32),
                ("trace_cap", C.c_int32), ("reserved", C.c_int32)]


def lib():
    """Load libdlmcol.so (never builds it; see paper_2109_05948_amd.build)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is missing: build it with "
                                  "`python -m paper_2109_05948_amd.build`")
            L = C.CDLL(LIB_PATH)
            P, I32, I64, U64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
            L.dlm_abi_version.restype = C.c_int
            L.dlm_last_error.restype = C.c_char_p
            L.dlm_graph_create.argtypes = [I32, P, P, P, C.c_uint32, P, C.POINTER(P)]
            L.dlm_graph_destroy.argtypes = [P]
            L.dlm_graph_info.argtypes = [P, C.POINTER(I32), C.POINTER(I64), C.POINTER(I32)]
            L.dlm_init_population.argtypes = [P, I32, I32, U64, I32, I32, P, P, P]
            L.dlm_tabu_workspace_bytes.argtypes = [P, C.POINTER(TabuParams), I32, C.POINTER(C.c_size_t)]
            L.dlm_tabu_batch.argtypes = [P, C.POINTER(TabuParams), I32, P, P, P, P, P, P, P, C.c_size_t, P]
            L.dlm_tabu_batch_static.argtypes = [P, C.POINTER(TabuParams), I32, P, P, P, P, P, P, P]
            L.dlm_evaluate.argtypes = [P, I32, P, I32, P, P, P]
            L.dlm_gpx_batch.argtypes = [P, I32, P, I32, P, I32, I32, U64, C.c_uint32, P, P]
            L.dlm_select.argtypes = [P, I32, I32, I32, U64, C.c_uint32, P, P, P]
            L.dlm_wvcp_batch.argtypes = [P, C.c_void_p, I32, P, P, P, P, P]
            L.dlm_scorer_create.argtypes = [I32, I32, I32, I32, I32, I32, P, C.POINTER(P)]
            L.dlm_scorer_destroy.argtypes = [P]
            L.dlm_scorer_num_params.argtypes = [P, C.POINTER(I64)]
            L.dlm_scorer_get_params.argtypes = [P, P, P]
            L.dlm_score_offspring.argtypes = [P, P, I32, P, P]
            L.dlm_scorer_grad.argtypes = [P, P, P, I32, P, P, P]
            L.dlm_scorer_train.argtypes = [P, P, P, I32, I32, I32, C.c_float, P, P]
            L.dlm_gather_rows.argtypes = [P, I32, I32, P, I32, P, P]
            L.dlm_standardize.argtypes = [P, I32, P, P]
            L.dlm_random_pairs.argtypes = [I32, U64, C.c_uint32, P, P]
            L.dlm_pop_update.argtypes = [P, P, P, P, I32, I32, P, P, P, P]
            L.dlm_multi_plan_create.argtypes = [P, I32, P, P, C.POINTER(P)]
            L.dlm_multi_plan_launch.argtypes = [P, P]
            L.dlm_multi_plan_info.argtypes = [P] + [C.POINTER(I32)] * 4
            L.dlm_multi_plan_destroy.argtypes = [P]
            L.dlm_multi_autotune.argtypes = [P, I32, I32, P, P, P]
            L.dlm_probe_lds_bandwidth.argtypes = [I32, C.POINTER(C.c_double), P]
            L.dlm_partition_distance.argtypes = [I32, I32, P, I32, P, I32, I32, P, I64, P, P]
            L.dlm_spacing_update.argtypes = [P, I32, P, I32, P, I64, I32, I32, P, P, P, P]
            L.dlm_gather_distances.argtypes = [P, I64, P, I32, P, I64, P]
            L.dlm_gather_pool.argtypes = [P, P, I32, P, P, I32, I32, P, I32, P, P, P]
            L.dlm_nearest.argtypes = [P, I64, I32, I32, P, P]
            L.dlm_select_groups.argtypes = [P, I32, I32, I32, U64, C.c_uint32, P, P]
            L.dlm_reduce_colours.argtypes = [P, I32, I32, I32, U64, C.c_uint32, P]
            L.dlm_invnet_create.argtypes = [I32, I32, I32, P, P, I32, C.POINTER(P)]
            L.dlm_invnet_destroy.argtypes = [P]
            L.dlm_invnet_num_params.argtypes = [P, C.POINTER(I64), C.POINTER(I64)]
            L.dlm_invnet_get_params.argtypes = [P, P, P]
            L.dlm_invnet_forward.argtypes = [P, P, I32, P, P]
            L.dlm_invnet_grad.argtypes = [P, P, P, I32, P, P, P]
            L.dlm_invnet_train.argtypes = [P, P, P, I32, I32, I32, C.c_float, P, P]
            L.dlm_wvcp_targets.argtypes = [P, I32, P, P, P]
            L.dlm_gemm_bf16.argtypes = [I32, P, I64, I32, P, I64, P, I64, I32, I32, I32, I32, I32, P, I64, P]
            for name in EXPORTS:
                getattr(L, name)
            _lib = L
    return _lib


def _check(fn: str, rc: int):
    if rc != DLM_OK:
        raise DlmError(fn, rc, lib().dlm_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data_as(C.c_void_p)
    return C.c_void_p(t.data_ptr())


def _dev(t: torch.Tensor, dtype, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    return t


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def abi_version() -> int:
    return int(lib().dlm_abi_version())


class Graph:
    """dlm_graph: a validated CSR graph resident in device memory."""

    def __init__(self, n: int, row_ptr, col_idx, weights=None, flags: int = 0, stream=None):
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        w = None if weights is None else np.ascontiguousarray(weights, dtype=np.int32)
        h = C.c_void_p()
        st = _stream(stream) if torch.cuda.is_available() else None
        _check("dlm_graph_create", lib().dlm_graph_create(n, _ptr(rp), _ptr(ci), _ptr(w), flags, st,
                                                          C.byref(h)))
        self._h = h
        self.n = int(n)
        self.weighted = w is not None

    @classmethod
    def from_csr(cls, g) -> "Graph":
        """From any object with n, row_ptr, col_idx and (optional) weights."""
        return cls(g.n, g.row_ptr, g.col_idx, getattr(g, "weights", None))

    @property
    def handle(self):
        return self._h

    def info(self) -> tuple[int, int, int]:
        n, nnz, md = C.c_int32(), C.c_int64(), C.c_int32()
        _check("dlm_graph_info", lib().dlm_graph_info(self._h, C.byref(n), C.byref(nnz), C.byref(md)))
        return n.value, nnz.value, md.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().dlm_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def init_population(graph: Graph, k: int, pop: int, seed: int, ind_base: int = 0,
                    mode: str = "random", colors: torch.Tensor | None = None,
                    k_used: torch.Tensor | None = None, stream=None):
    """dlm_init_population -> (colors int16 [pop, n], k_used int32 [pop])."""
    dev = torch.device("cuda", torch.cuda.current_device())
    if colors is None:
        colors = torch.empty((pop, graph.n), dtype=torch.int16, device=dev)
    if k_used is None:
        k_used = torch.empty((pop,), dtype=torch.int32, device=dev)
    _dev(colors, torch.int16, "colors")
    _dev(k_used, torch.int32, "k_used")
    _check("dlm_init_population",
           lib().dlm_init_population(graph.handle, k, pop, seed & (2**64 - 1), ind_base,
                                     INIT_MODES[mode], _ptr(colors), _ptr(k_used), _stream(stream)))
    return colors, k_used


def _tabu_params(k, max_iters, seed, ind_base, ten_num, ten_den, ten_rand, block, table, trace_cap):
    return TabuParams(k, max_iters, ten_num, ten_den, ten_rand, ind_base, seed & (2**64 - 1),
                      block, TABLES[table], trace_cap, 0)


def tabu_workspace_bytes(graph: Graph, pop: int, k: int, max_iters: int, seed: int = 0,
                         ind_base: int = 0, ten_num: int = 6, ten_den: int = 10, ten_rand: int = 10,
                         block: int = 0, table: str = "auto", trace_cap: int = 0) -> int:
    """dlm_tabu_workspace_bytes: device scratch a dlm_tabu_batch call needs."""
    prm = _tabu_params(k, max_iters, seed, ind_base, ten_num, ten_den, ten_rand, block, table, trace_cap)
    out = C.c_size_t()
    _check("dlm_tabu_workspace_bytes",
           lib().dlm_tabu_workspace_bytes(graph.handle, C.byref(prm), pop, C.byref(out)))
    return int(out.value)


def tabu_batch(graph: Graph, colors: torch.Tensor, k: int, max_iters: int, seed: int,
               ind_base: int = 0, ten_num: int = 6, ten_den: int = 10, ten_rand: int = 10,
               block: int = 0, table: str = "auto", stats: bool = True, hashes: bool = True,
               trace_cap: int = 0, out: dict | None = None, workspace: torch.Tensor | None = None,
               stream=None) -> dict:
    """dlm_tabu_batch on every row of ``colors`` (modified in place to the best colouring).

    The device workspace is a torch tensor: ``workspace`` if given (uint8, at
    least dlm_tabu_workspace_bytes), else one taken from torch's allocator
    for this call."""
    _dev(colors, torch.int16, "colors")
    pop = colors.shape[0]
    if colors.dim() != 2 or colors.shape[1] != graph.n:
        raise ValueError(f"colors must be [pop, {graph.n}]")
    dev = colors.device
    o = out if out is not None else {}
    if "f_best" not in o:
        o["f_best"] = torch.empty(pop, dtype=torch.int32, device=dev)
        o["iters"] = torch.empty(pop, dtype=torch.int32, device=dev)
        o["stats"] = torch.empty((pop, NSTATS), dtype=torch.int64, device=dev) if stats else None
        o["hash"] = torch.empty(pop, dtype=torch.int64, device=dev) if hashes else None
        o["trace"] = (torch.empty((pop, trace_cap, 2), dtype=torch.int32, device=dev)
                      if trace_cap else None)
    prm = _tabu_params(k, max_iters, seed, ind_base, ten_num, ten_den, ten_rand, block, table, trace_cap)
    if workspace is None:
        need = C.c_size_t()
        _check("dlm_tabu_workspace_bytes",
               lib().dlm_tabu_workspace_bytes(graph.handle, C.byref(prm), pop, C.byref(need)))
        workspace = torch.empty(need.value, dtype=torch.uint8, device=dev) if need.value else None
    if workspace is not None:
        _dev(workspace, torch.uint8, "workspace")
    ws_bytes = workspace.numel() if workspace is not None else 0
    _check("dlm_tabu_batch",
           lib().dlm_tabu_batch(graph.handle, C.byref(prm), pop, _ptr(colors), _ptr(o["f_best"]),
                                _ptr(o["iters"]), _ptr(o.get("stats")), _ptr(o.get("hash")),
                                _ptr(o.get("trace")), _ptr(workspace), ws_bytes, _stream(stream)))
    o["colors"] = colors
    return o


STATIC_SCRATCH_BYTES = 64 << 20  # DLM_STATIC_SCRATCH_BYTES


def tabu_batch_static(graph: Graph, colors: torch.Tensor, k: int, max_iters: int, seed: int, out: dict,
                      ind_base: int = 0, ten_num: int = 6, ten_den: int = 10, ten_rand: int = 10,
                      block: int = 0, table: str = "auto", trace_cap: int = 0, stream=None) -> dict:
    """dlm_tabu_batch_static: dlm_tabu_batch with the library's fixed device
    scratch as its workspace.  Nothing is allocated here either: ``out``
    holds the caller's f_best, iters and (or None) stats, hash, trace tensors."""
    _dev(colors, torch.int16, "colors")
    pop = colors.shape[0]
    if colors.dim() != 2 or colors.shape[1] != graph.n:
        raise ValueError(f"colors must be [pop, {graph.n}]")
    prm = _tabu_params(k, max_iters, seed, ind_base, ten_num, ten_den, ten_rand, block, table, trace_cap)
    _check("dlm_tabu_batch_static",
           lib().dlm_tabu_batch_static(graph.handle, C.byref(prm), pop, _ptr(colors), _ptr(out["f_best"]),
                                       _ptr(out["iters"]), _ptr(out.get("stats")), _ptr(out.get("hash")),
                                       _ptr(out.get("trace")), _stream(stream)))
    out["colors"] = colors
    return out


def evaluate(graph: Graph, colors: torch.Tensor, k: int, weighted: bool = False, stream=None):
    """dlm_evaluate -> (conflicts int32 [count], wscore int32 [count] or None)."""
    _dev(colors, torch.int16, "colors")
    cnt = colors.shape[0]
    conf = torch.empty(cnt, dtype=torch.int32, device=colors.device)
    ws = torch.empty(cnt, dtype=torch.int32, device=colors.device) if weighted else None
    _check("dlm_evaluate", lib().dlm_evaluate(graph.handle, k, _ptr(colors), cnt, _ptr(conf),
                                              _ptr(ws), _stream(stream)))
    return conf, ws


def gpx_batch(graph: Graph, k: int, parents: torch.Tensor, pairs: torch.Tensor, per_pair: int,
              seed: int, child_base: int = 0, children: torch.Tensor | None = None, stream=None):
    """dlm_gpx_batch -> children int16 [npairs * per_pair, n]."""
    _dev(parents, torch.int16, "parents")
    _dev(pairs, torch.int32, "pairs")
    npairs = pairs.shape[0]
    if children is None:
        children = torch.empty((npairs * per_pair, graph.n), dtype=torch.int16,
                               device=parents.device)
    _dev(children, torch.int16, "children")
    _check("dlm_gpx_batch",
           lib().dlm_gpx_batch(graph.handle, k, _ptr(parents), parents.shape[0], _ptr(pairs),
                               npairs, per_pair, seed & (2**64 - 1), child_base & 0xffffffff,
                               _ptr(children), _stream(stream)))
    return children


def select(scores: torch.Tensor | None, count: int, keep: int, mode: str = "top", seed: int = 0,
           gen: int = 0, stream=None) -> torch.Tensor:
    """dlm_select -> int32 [keep] indices in rank order ("top" or "random")."""
    dev = scores.device if scores is not None else torch.device("cuda", torch.cuda.current_device())
    if scores is not None:
        _dev(scores, torch.float32, "scores")
    out = torch.empty(keep, dtype=torch.int32, device=dev)
    ws = torch.empty(max(count, 1), dtype=torch.int64, device=dev)
    _check("dlm_select", lib().dlm_select(_ptr(scores), count, keep, {"top": 0, "random": 1}[mode],
                                          seed & (2**64 - 1), gen & 0xffffffff, _ptr(out), _ptr(ws),
                                          _stream(stream)))
    return out


class WvcpParams(C.Structure):
    _fields_ = [("k", C.c_int32), ("iters_per_round", C.c_int32), ("rounds", C.c_int32),
                ("ten_rand", C.c_int32), ("frz_num", C.c_int32), ("frz_den", C.c_int32),
                ("shift", C.c_int32), ("ind_base", C.c_int32), ("seed", C.c_uint64),
                ("block", C.c_int32), ("reserved", C.c_int32)]


def wvcp_batch(graph: Graph, colors: torch.Tensor, k: int, iters_per_round: int, rounds: int,
               seed: int, ind_base: int = 0, ten_rand: int = 10, frz_num: int = 2,
               frz_den: int = 10, shift: int = 10, block: int = 0, stream=None) -> dict:
    """dlm_wvcp_batch on every row of ``colors`` (in place: best legal colouring)."""
    _dev(colors, torch.int16, "colors")
    pop = colors.shape[0]
    if colors.dim() != 2 or colors.shape[1] != graph.n:
        raise ValueError(f"colors must be [pop, {graph.n}]")
    dev = colors.device
    o = {"best_legal": torch.empty(pop, dtype=torch.int32, device=dev),
         "stats": torch.empty((pop, NSTATS), dtype=torch.int64, device=dev),
         "hash": torch.empty(pop, dtype=torch.int64, device=dev)}
    prm = WvcpParams(k, iters_per_round, rounds, ten_rand, frz_num, frz_den, shift, ind_base,
                     seed & (2**64 - 1), block, 0)
    _check("dlm_wvcp_batch",
           lib().dlm_wvcp_batch(graph.handle, C.byref(prm), pop, _ptr(colors),
                                _ptr(o["best_legal"]), _ptr(o["stats"]), _ptr(o["hash"]),
                                _stream(stream)))
    o["colors"] = colors
    return o


SCORER_NAMES = ("W1", "b1", "W2", "b2", "W3", "b3", "w4", "b4")


class Scorer:
    """dlm_scorer: per-class MLP offspring scorer (FP32 master, BF16 working copy, Adam)."""

    def __init__(self, n: int, k: int, params: dict, max_batch: int = 1024,
                 widths: tuple = (256, 128, 64)):
        flat = np.concatenate([np.ascontiguousarray(params[nm], dtype=np.float32).reshape(-1)
                               for nm in SCORER_NAMES])
        h = C.c_void_p()
        _check("dlm_scorer_create", lib().dlm_scorer_create(n, k, *widths, max_batch, _ptr(flat),
                                                            C.byref(h)))
        self._h, self.n, self.k, self.max_batch = h, n, k, max_batch
        self.shapes = {nm: np.asarray(params[nm]).shape for nm in SCORER_NAMES}
        cnt = C.c_int64()
        _check("dlm_scorer_num_params", lib().dlm_scorer_num_params(h, C.byref(cnt)))
        self.num_params = cnt.value
        assert self.num_params == flat.size

    def unpack(self, flat: np.ndarray) -> dict:
        out, o = {}, 0
        for nm in SCORER_NAMES:
            sz = int(np.prod(self.shapes[nm]))
            out[nm] = flat[o:o + sz].reshape(self.shapes[nm])
            o += sz
        return out

    def params(self, stream=None) -> dict:
        buf = torch.empty(self.num_params, dtype=torch.float32, device="cuda")
        _check("dlm_scorer_get_params", lib().dlm_scorer_get_params(self._h, _ptr(buf), _stream(stream)))
        return self.unpack(buf.cpu().numpy())

    def score(self, colors: torch.Tensor, out: torch.Tensor | None = None, stream=None):
        """dlm_score_offspring -> float32 [count]."""
        _dev(colors, torch.int16, "colors")
        cnt = colors.shape[0]
        out = out if out is not None else torch.empty(cnt, dtype=torch.float32, device=colors.device)
        _check("dlm_score_offspring", lib().dlm_score_offspring(self._h, _ptr(colors), cnt, _ptr(out),
                                                                _stream(stream)))
        return out

    def grad(self, colors: torch.Tensor, targets: torch.Tensor, stream=None):
        """dlm_scorer_grad -> (flat FP32 gradient of the mean squared error, loss)."""
        _dev(colors, torch.int16, "colors")
        _dev(targets, torch.float32, "targets")
        g = torch.empty(self.num_params, dtype=torch.float32, device=colors.device)
        loss = torch.empty(1, dtype=torch.float32, device=colors.device)
        _check("dlm_scorer_grad", lib().dlm_scorer_grad(self._h, _ptr(colors), _ptr(targets),
                                                        colors.shape[0], _ptr(g), _ptr(loss),
                                                        _stream(stream)))
        return g, loss

    def train(self, colors: torch.Tensor, targets: torch.Tensor, batch: int, epochs: int,
              lr: float = 1e-3, stream=None) -> torch.Tensor:
        """dlm_scorer_train -> per-step losses."""
        _dev(colors, torch.int16, "colors")
        _dev(targets, torch.float32, "targets")
        cnt = colors.shape[0]
        steps = epochs * ((cnt + batch - 1) // batch)
        loss = torch.empty(max(steps, 1), dtype=torch.float32, device=colors.device)
        _check("dlm_scorer_train", lib().dlm_scorer_train(self._h, _ptr(colors), _ptr(targets), cnt,
                                                          batch, epochs, C.c_float(lr), _ptr(loss),
                                                          _stream(stream)))
        return loss[:steps]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().dlm_scorer_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def invnet_names(widths) -> tuple[list[str], list[str]]:
    """Names of the packed dlm_invnet layout: the trainables per layer (Lambda
    L, Gamma G, beta b, and for hidden layers the scale g and shift m), then
    the running mean rm and variance rv of every hidden layer."""
    train, run = [], []
    for j in range(len(widths)):
        train += [f"L{j}", f"G{j}", f"b{j}"]
        if j < len(widths) - 1:
            train += [f"g{j}", f"m{j}"]
            run += [f"rm{j}", f"rv{j}"]
    return train, run


class InvNet:
    """dlm_invnet: the colour-invariant network (FP32 trainables, BF16 GEMM
    operands, invariant batch normalisation, Adam)."""

    def __init__(self, n: int, k: int, widths, params: dict, max_batch: int = 64):
        self.widths = [int(w) for w in widths]
        self.train_names, self.run_names = invnet_names(self.widths)
        names = self.train_names + self.run_names
        flat = np.concatenate([np.ascontiguousarray(params[nm], dtype=np.float32).reshape(-1)
                               for nm in names])
        w = np.asarray(self.widths, dtype=np.int32)
        h = C.c_void_p()
        _check("dlm_invnet_create", lib().dlm_invnet_create(n, k, len(self.widths), _ptr(w), _ptr(flat),
                                                            max_batch, C.byref(h)))
        self._h, self.n, self.k, self.max_batch = h, n, k, max_batch
        self.shapes = {nm: np.asarray(params[nm]).shape for nm in names}
        tr, rn = C.c_int64(), C.c_int64()
        _check("dlm_invnet_num_params", lib().dlm_invnet_num_params(h, C.byref(tr), C.byref(rn)))
        self.num_trainable, self.num_running = tr.value, rn.value
        assert self.num_trainable + self.num_running == flat.size

    def unpack(self, flat: np.ndarray, names=None) -> dict:
        out, o = {}, 0
        for nm in (names if names is not None else self.train_names + self.run_names):
            sz = int(np.prod(self.shapes[nm]))
            out[nm] = flat[o:o + sz].reshape(self.shapes[nm])
            o += sz
        return out

    def params(self, stream=None) -> dict:
        buf = torch.empty(self.num_trainable + self.num_running, dtype=torch.float32, device="cuda")
        _check("dlm_invnet_get_params", lib().dlm_invnet_get_params(self._h, _ptr(buf), _stream(stream)))
        return self.unpack(buf.cpu().numpy())

    def forward(self, colors: torch.Tensor, out: torch.Tensor | None = None, stream=None):
        """dlm_invnet_forward (evaluation) -> float32 [count]."""
        _dev(colors, torch.int16, "colors")
        cnt = colors.shape[0]
        out = out if out is not None else torch.empty(cnt, dtype=torch.float32, device=colors.device)
        _check("dlm_invnet_forward", lib().dlm_invnet_forward(self._h, _ptr(colors), cnt, _ptr(out),
                                                              _stream(stream)))
        return out

    score = forward  # the scorer interface of the memetic loop

    def grad(self, colors: torch.Tensor, targets: torch.Tensor, stream=None):
        """dlm_invnet_grad -> (flat FP32 gradient of the batch MSE, loss)."""
        _dev(colors, torch.int16, "colors")
        _dev(targets, torch.float32, "targets")
        g = torch.empty(self.num_trainable, dtype=torch.float32, device=colors.device)
        loss = torch.empty(1, dtype=torch.float32, device=colors.device)
        _check("dlm_invnet_grad", lib().dlm_invnet_grad(self._h, _ptr(colors), _ptr(targets),
                                                        colors.shape[0], _ptr(g), _ptr(loss),
                                                        _stream(stream)))
        return g, loss

    def train(self, colors: torch.Tensor, targets: torch.Tensor, batch: int, epochs: int,
              lr: float = 1e-3, stream=None) -> torch.Tensor:
        """dlm_invnet_train -> per-step losses."""
        _dev(colors, torch.int16, "colors")
        _dev(targets, torch.float32, "targets")
        cnt = colors.shape[0]
        steps = epochs * ((cnt + batch - 1) // batch)
        loss = torch.empty(max(steps, 1), dtype=torch.float32, device=colors.device)
        _check("dlm_invnet_train", lib().dlm_invnet_train(self._h, _ptr(colors), _ptr(targets), cnt,
                                                          batch, epochs, C.c_float(lr), _ptr(loss),
                                                          _stream(stream)))
        return loss[:steps]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().dlm_invnet_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gather_rows(src: torch.Tensor, idx: torch.Tensor, out: torch.Tensor | None = None, stream=None):
    """dlm_gather_rows -> int16 [len(idx), n]."""
    _dev(src, torch.int16, "src")
    _dev(idx, torch.int32, "idx")
    out = out if out is not None else torch.empty((idx.shape[0], src.shape[1]), dtype=torch.int16,
                                                  device=src.device)
    _check("dlm_gather_rows", lib().dlm_gather_rows(_ptr(src), src.shape[0], src.shape[1], _ptr(idx),
                                                    idx.shape[0], _ptr(out), _stream(stream)))
    return out


def standardize(f: torch.Tensor, out: torch.Tensor | None = None, stream=None):
    """dlm_standardize -> float32 (f - mean) / std."""
    _dev(f, torch.int32, "f")
    out = out if out is not None else torch.empty(f.shape[0], dtype=torch.float32, device=f.device)
    _check("dlm_standardize", lib().dlm_standardize(_ptr(f), f.shape[0], _ptr(out), _stream(stream)))
    return out


def wvcp_targets(f: torch.Tensor, out: torch.Tensor | None = None, stream=None):
    """dlm_wvcp_targets -> (targets int32 [count], device flag int32 [1]:
    1 if some search met a legal colouring)."""
    _dev(f, torch.int32, "f")
    out = out if out is not None else torch.empty_like(f)
    flag = torch.empty(1, dtype=torch.int32, device=f.device)
    _check("dlm_wvcp_targets", lib().dlm_wvcp_targets(_ptr(f), f.numel(), _ptr(out), _ptr(flag), _stream(stream)))
    return out, flag


def random_pairs(pop: int, seed: int, gen: int, out: torch.Tensor | None = None, stream=None):
    """dlm_random_pairs -> int32 [pop, 2]."""
    out = out if out is not None else torch.empty((pop, 2), dtype=torch.int32, device="cuda")
    _check("dlm_random_pairs", lib().dlm_random_pairs(pop, seed & (2**64 - 1), gen & 0xffffffff,
                                                      _ptr(out), _stream(stream)))
    return out


def pop_update(parents: torch.Tensor, f_parents: torch.Tensor, offspring: torch.Tensor,
               f_offspring: torch.Tensor, out=None, f_out=None, stream=None):
    """dlm_pop_update -> (colours [pop, n], scores [pop]) of the best pop of both."""
    pop, n = parents.shape
    for t, nm in ((parents, "parents"), (offspring, "offspring")):
        _dev(t, torch.int16, nm)
    for t, nm in ((f_parents, "f_parents"), (f_offspring, "f_offspring")):
        _dev(t, torch.int32, nm)
    out = out if out is not None else torch.empty_like(parents)
    f_out = f_out if f_out is not None else torch.empty_like(f_parents)
    ws = torch.empty(3 * pop, dtype=torch.int64, device=parents.device)
    _check("dlm_pop_update", lib().dlm_pop_update(_ptr(parents), _ptr(f_parents), _ptr(offspring),
                                                  _ptr(f_offspring), pop, n, _ptr(out), _ptr(f_out),
                                                  _ptr(ws), _stream(stream)))
    return out, f_out


def partition_distance(a: torch.Tensor, k: int, b: torch.Tensor | None = None, out: torch.Tensor | None = None,
                       upper_only: bool = False, stream=None):
    """dlm_partition_distance -> int32 [len(a), len(b)]; b None: the
    triangle form over the rows of a (symmetric, zero diagonal; with
    upper_only the strict lower triangle is left as it was).  ``out`` may be
    a row-strided view (e.g. a block of a pool matrix)."""
    _dev(a, torch.int16, "a")
    tri = b is None
    b = a if tri else b
    _dev(b, torch.int16, "b")
    if a.dim() != 2 or b.dim() != 2 or a.shape[1] != b.shape[1]:
        raise ValueError("a and b must be [rows, n] with the same n")
    na, nb, n = a.shape[0], b.shape[0], a.shape[1]
    if out is None:
        out = torch.empty((na, nb), dtype=torch.int32, device=a.device)
    if out.dtype != torch.int32 or out.shape != (na, nb) or out.stride(1) != 1:
        raise ValueError(f"out must be int32 [{na}, {nb}] with unit column stride")
    ws = torch.empty(((k + 2) * (na + nb) + 1) // 2 + 1, dtype=torch.int32, device=a.device)
    _check("dlm_partition_distance", lib().dlm_partition_distance(
        n, k, _ptr(a), na, _ptr(b), nb, (2 if upper_only else 1) if tri else 0, _ptr(out), out.stride(0), _ptr(ws),
        _stream(stream)))
    return out


def spacing_update(fa: torch.Tensor, fb: torch.Tensor, dist: torch.Tensor, keep: int, spacing: int,
                   stream=None):
    """dlm_spacing_update -> (pick int32 [keep], n_spaced int32 [1]); dist is
    the pool's [na + nb, >= na + nb] matrix (its upper triangle is read)."""
    _dev(fa, torch.int32, "fa")
    _dev(fb, torch.int32, "fb")
    _dev(dist, torch.int32, "dist")
    total = fa.shape[0] + fb.shape[0]
    if dist.shape[0] < total or dist.shape[1] < total or dist.stride(1) != 1:
        raise ValueError(f"dist must cover the pool of {total}")
    pick = torch.empty(keep, dtype=torch.int32, device=fa.device)
    nsp = torch.empty(1, dtype=torch.int32, device=fa.device)
    ws = torch.empty(max(total, 1), dtype=torch.int32, device=fa.device)
    _check("dlm_spacing_update", lib().dlm_spacing_update(
        _ptr(fa), fa.shape[0], _ptr(fb), fb.shape[0], _ptr(dist), dist.stride(0), keep, spacing, _ptr(pick),
        _ptr(nsp), _ptr(ws), _stream(stream)))
    return pick, nsp


def gather_distances(dist: torch.Tensor, idx: torch.Tensor, out: torch.Tensor | None = None, stream=None):
    """dlm_gather_distances -> int32 [len(idx), len(idx)] (may be a strided view)."""
    _dev(dist, torch.int32, "dist")
    _dev(idx, torch.int32, "idx")
    c = idx.shape[0]
    out = out if out is not None else torch.empty((c, c), dtype=torch.int32, device=dist.device)
    if out.shape != (c, c) or out.stride(1) != 1:
        raise ValueError(f"out must be [{c}, {c}] with unit column stride")
    _check("dlm_gather_distances", lib().dlm_gather_distances(
        _ptr(dist), dist.stride(0), _ptr(idx), c, _ptr(out), out.stride(0), _stream(stream)))
    return out


def gather_pool(ra: torch.Tensor, fa: torch.Tensor, rb: torch.Tensor, fb: torch.Tensor, pick: torch.Tensor,
                stream=None):
    """dlm_gather_pool -> (rows int16 [len(pick), n], scores int32 [len(pick)])."""
    for t, nm in ((ra, "ra"), (rb, "rb")):
        _dev(t, torch.int16, nm)
    for t, nm in ((fa, "fa"), (fb, "fb"), (pick, "pick")):
        _dev(t, torch.int32, nm)
    n = ra.shape[1]
    out = torch.empty((pick.shape[0], n), dtype=torch.int16, device=ra.device)
    fout = torch.empty(pick.shape[0], dtype=torch.int32, device=ra.device)
    _check("dlm_gather_pool", lib().dlm_gather_pool(
        _ptr(ra), _ptr(fa), ra.shape[0], _ptr(rb), _ptr(fb), rb.shape[0], n, _ptr(pick), pick.shape[0],
        _ptr(out), _ptr(fout), _stream(stream)))
    return out, fout


def select_groups(scores: torch.Tensor | None, groups: int, K: int, mode: str = "top", seed: int = 0,
                  gen: int = 0, stream=None):
    """dlm_select_groups -> int32 [groups]: one child index per group of K."""
    m = {"top": 0, "random": 1}[mode]
    if m == 0:
        _dev(scores, torch.float32, "scores")
        if scores.shape[0] < groups * K:
            raise ValueError("scores shorter than groups * K")
    out = torch.empty(groups, dtype=torch.int32, device="cuda")
    _check("dlm_select_groups", lib().dlm_select_groups(_ptr(scores) if m == 0 else None, groups, K, m,
                                                        seed & (2**64 - 1), gen & 0xffffffff, _ptr(out),
                                                        _stream(stream)))
    return out


def reduce_colours(colors: torch.Tensor, k: int, seed: int, step: int, stream=None):
    """dlm_reduce_colours: k -> k - 1 colours, in place on colors (int16 [pop, n])."""
    _dev(colors, torch.int16, "colors")
    _check("dlm_reduce_colours", lib().dlm_reduce_colours(_ptr(colors), colors.shape[0], colors.shape[1], k,
                                                          seed & (2**64 - 1), step & 0xffffffff, _stream(stream)))
    return colors


def nearest(dist: torch.Tensor, K: int, p: int | None = None, stream=None):
    """dlm_nearest -> int32 [p, K] (p defaults to dist.shape[0])."""
    _dev(dist, torch.int32, "dist")
    p = dist.shape[0] if p is None else p
    if dist.stride(1) != 1:
        raise ValueError("dist must have unit column stride")
    out = torch.empty((p, K), dtype=torch.int32, device=dist.device)
    _check("dlm_nearest", lib().dlm_nearest(_ptr(dist), dist.stride(0), p, K, _ptr(out), _stream(stream)))
    return out


class MultiItem(C.Structure):
    _fields_ = [("g", C.c_void_p), ("k", C.c_int32), ("max_iters", C.c_int32), ("pop", C.c_int32),
                ("ind_base", C.c_int32), ("ten_num", C.c_int32), ("ten_den", C.c_int32),
                ("ten_rand", C.c_int32), ("reserved", C.c_int32), ("seed", C.c_uint64),
                ("colors_dev", C.c_void_p), ("f_best_dev", C.c_void_p), ("iters_dev", C.c_void_p),
                ("stats_dev", C.c_void_p), ("hash_dev", C.c_void_p)]


class MultiConfig(C.Structure):
    _fields_ = [("block", C.c_int32), ("lds_budget", C.c_int32)]


class MultiBatch:
    """An uneven batch: per graph a population, searched by one persistent hipGraph launch.

    ``jobs`` is a list of dicts with keys graph (Graph), colors (int16 device
    tensor [pop, n]), k, iters, seed and optionally ind_base, ten_num,
    ten_den, ten_rand.  Outputs (f_best, iters, stats, hash) are allocated
    here and refreshed by every ``launch``.
    """

    def __init__(self, jobs: list, block: int = 0, lds_budget: int = 0, stream=None):
        self.jobs = jobs
        self._items = (MultiItem * len(jobs))()
        for i, j in enumerate(jobs):
            col = _dev(j["colors"], torch.int16, "colors")
            pop = col.shape[0]
            j.setdefault("f_best", torch.empty(pop, dtype=torch.int32, device=col.device))
            j.setdefault("iters_out", torch.empty(pop, dtype=torch.int32, device=col.device))
            j.setdefault("stats", torch.empty((pop, NSTATS), dtype=torch.int64, device=col.device))
            j.setdefault("hash", torch.empty(pop, dtype=torch.int64, device=col.device))
            self._items[i] = MultiItem(
                j["graph"].handle.value, j["k"], j["iters"], pop, j.get("ind_base", 0),
                j.get("ten_num", 6), j.get("ten_den", 10), j.get("ten_rand", 10), 0,
                j["seed"] & (2**64 - 1), col.data_ptr(), j["f_best"].data_ptr(),
                j["iters_out"].data_ptr(), j["stats"].data_ptr(), j["hash"].data_ptr())
        self.config = MultiConfig(block, lds_budget)
        h = C.c_void_p()
        _check("dlm_multi_plan_create", lib().dlm_multi_plan_create(self._items, len(jobs),
                                                                    C.byref(self.config),
                                                                    _stream(stream), C.byref(h)))
        self._h = h

    @classmethod
    def autotune(cls, jobs: list, calib_iters: int = 2000, stream=None):
        """dlm_multi_autotune -> (best (block, lds_budget), rates of all 12 candidates)."""
        items = (MultiItem * len(jobs))()
        keep = []
        for i, j in enumerate(jobs):
            col = _dev(j["colors"], torch.int16, "colors")
            pop = col.shape[0]
            scratch = [torch.empty(pop, dtype=torch.int32, device=col.device) for _ in range(2)]
            keep.append(scratch)
            items[i] = MultiItem(j["graph"].handle.value, j["k"], j["iters"], pop, j.get("ind_base", 0),
                                 j.get("ten_num", 6), j.get("ten_den", 10), j.get("ten_rand", 10), 0,
                                 j["seed"] & (2**64 - 1), col.data_ptr(), scratch[0].data_ptr(),
                                 scratch[1].data_ptr(), None, None)
        best = MultiConfig()
        rates = np.zeros(12, dtype=np.float32)
        _check("dlm_multi_autotune", lib().dlm_multi_autotune(items, len(jobs), calib_iters,
                                                              C.byref(best), _ptr(rates),
                                                              _stream(stream)))
        return (best.block, best.lds_budget), rates

    def info(self) -> dict:
        g, l, ng, t = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check("dlm_multi_plan_info", lib().dlm_multi_plan_info(self._h, C.byref(g), C.byref(l),
                                                                C.byref(ng), C.byref(t)))
        return {"grid": g.value, "lds_bytes": l.value, "graphs_on_device_table": ng.value,
                "items": t.value}

    def launch(self, stream=None):
        _check("dlm_multi_plan_launch", lib().dlm_multi_plan_launch(self._h, _stream(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().dlm_multi_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gemm_bf16(a: torch.Tensor, b: torch.Tensor, m: int, n: int, k: int, a_kcontig: bool, b_kcontig: bool,
              sa: int | None = None, sb: int | None = None, out: torch.Tensor | None = None, ldc: int | None = None,
              tile: int = 0, splits: int = 0, workspace: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """dlm_gemm_bf16: C[m][n] = sum_k A(m, k) B(k, n) in FP32 from BF16 (or
    raw int16) operands.  A(m, k) = a[m sa + k] if a_kcontig else a[k sa + m];
    B(k, n) = b[n sb + k] if b_kcontig else b[k sb + n]; the pitches default
    to the contiguous extents.  ``workspace`` (any contiguous CUDA tensor)
    holds split-K partials; a forced ``splits`` > 1 without one gets a fresh
    buffer.  Returns out (float32 [m][ldc])."""
    for t, nm in ((a, "a"), (b, "b")):
        if t.dtype not in (torch.bfloat16, torch.int16) or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{nm} must be a contiguous bfloat16 or int16 CUDA tensor")
    sa = sa if sa is not None else (k if a_kcontig else m)
    sb = sb if sb is not None else (k if b_kcontig else n)
    ldc = ldc if ldc is not None else n
    if out is None:
        out = torch.empty((m, ldc), dtype=torch.float32, device=a.device)
    _dev(out, torch.float32, "out")
    if out.numel() < m * ldc:
        raise ValueError("out is smaller than m * ldc")
    if workspace is None and splits > 1:
        workspace = torch.empty(splits * m * n, dtype=torch.float32, device=a.device)
    wptr, wbytes = (None, 0) if workspace is None else (_ptr(workspace), workspace.numel() * workspace.element_size())
    _check("dlm_gemm_bf16", lib().dlm_gemm_bf16(int(a_kcontig), _ptr(a), sa, int(b_kcontig), _ptr(b), sb, _ptr(out),
                                                ldc, m, n, k, tile, splits, wptr, wbytes, _stream(stream)))
    return out


def probe_lds_bandwidth(rounds: int = 2000, stream=None) -> float:
    """dlm_probe_lds_bandwidth -> sustained device LDS read bandwidth (bytes/s)."""
    out = C.c_double()
    _check("dlm_probe_lds_bandwidth", lib().dlm_probe_lds_bandwidth(rounds, C.byref(out), _stream(stream)))
    return out.value

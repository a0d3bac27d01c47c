"""Exact connected-component labelling on AMD Instinct MI355X (gfx950).

Thin ctypes binding over ``libccmi.so`` (C ABI declared in ``include/cc.h``).
This module only marshals arguments: torch tensors provide device memory and
the current HIP stream; every step of the computation runs in the library's
HIP kernels.  If the library is not built the calls raise -- there is no CPU
fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import math
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libccmi.so")

ROUTE_AUTO, ROUTE_HEURISTIC, ROUTE_ROUTER, ROUTE_SV, ROUTE_BFS_SV, ROUTE_SV_THETA = range(6)
R0_BFS_SV, R1_SV, R2_SV_THETA = 0, 1, 2
ROUTE_NAMES = {R0_BFS_SV: "bfs+sv", R1_SV: "sv", R2_SV_THETA: "sv-theta"}
KERNEL_CLASSES = ["sv_pass", "sv_shortcut", "sv_finalize", "degree", "hist", "csr", "bfs", "filter"]
_ROUTE_ARG = {None: ROUTE_AUTO, "auto": ROUTE_AUTO, "heuristic": ROUTE_HEURISTIC, "router": ROUTE_ROUTER,
              "sv": ROUTE_SV, "bfs+sv": ROUTE_BFS_SV, "bfs": ROUTE_BFS_SV, "sv-theta": ROUTE_SV_THETA}

ROUTER_NPARAMS = 64 * 66 + 64 + 64 * 64 + 64 + 3 * 64 + 3
ROUTER_NFEATURES = 66

CC_OK, CC_EINVAL, CC_ERANGE, CC_ENOMEM, CC_EHIP, CC_EINTERNAL, CC_ENOROUTER = 0, -1, -2, -3, -4, -5, -6
_ERRNAMES = {-1: "CC_EINVAL", -2: "CC_ERANGE", -3: "CC_ENOMEM", -4: "CC_EHIP", -5: "CC_EINTERNAL",
             -6: "CC_ENOROUTER"}


class CCError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


SCRATCH_CACHED, SCRATCH_POOL = 0, 1
_SCRATCH_ARG = {None: SCRATCH_CACHED, "cached": SCRATCH_CACHED, "pool": SCRATCH_POOL}


class Options(ctypes.Structure):
    _fields_ = [("route", ctypes.c_int32), ("max_passes", ctypes.c_int32), ("tau", ctypes.c_double),
                ("theta", ctypes.c_double), ("profile", ctypes.c_int32), ("scratch", ctypes.c_int32),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_int64),
                ("check", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


class Stats(ctypes.Structure):
    _fields_ = [("route", ctypes.c_int32), ("sv_passes", ctypes.c_int32), ("bfs_levels", ctypes.c_int32),
                ("bfs_bottom_up_levels", ctypes.c_int32), ("bfs_seed", ctypes.c_int32),
                ("bfs_label", ctypes.c_int32), ("bfs_visited", ctypes.c_int64),
                ("bfs_edges_examined", ctypes.c_int64), ("edges_after_filter", ctypes.c_int64),
                ("max_degree", ctypes.c_int64), ("ks_statistic", ctypes.c_double), ("ks_alpha", ctypes.c_double),
                ("ks_dmin", ctypes.c_int64), ("router_logits", ctypes.c_float * 3), ("sv_deep_rounds", ctypes.c_int32),
                ("active_edges", ctypes.c_int64 * 64), ("hooks_total", ctypes.c_int64),
                ("ms_predict", ctypes.c_double), ("ms_csr", ctypes.c_double), ("ms_bfs", ctypes.c_double),
                ("ms_filter", ctypes.c_double), ("ms_sv", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("algorithmic_bytes", ctypes.c_double), ("kernel_ms", ctypes.c_double * 8),
                ("kernel_launches", ctypes.c_int32 * 8), ("kernel_bytes", ctypes.c_double * 8),
                ("sv_atomics", ctypes.c_int64), ("sv_chase_reads", ctypes.c_int64), ("giant_dropped", ctypes.c_int64),
                ("check_flags", ctypes.c_int32), ("check_pass_limit", ctypes.c_int32), ("sv_hubs", ctypes.c_int32)]

    def to_dict(self) -> dict:
        d = {}
        for name, _ in self._fields_:
            if name.startswith("reserved"):
                continue
            val = getattr(self, name)
            if name == "active_edges":
                val = [int(x) for x in val][: max(0, min(self.sv_passes, 64))]
            elif name in ("router_logits", "kernel_ms", "kernel_bytes"):
                val = [float(x) for x in val]
            elif name == "kernel_launches":
                val = [int(x) for x in val]
            d[name] = val
        d["route_name"] = ROUTE_NAMES.get(self.route, "none")
        return d


class TupleStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("sorts", ctypes.c_int32), ("passes_per_sort", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("tuples", ctypes.c_int64), ("ms_sort", ctypes.c_double),
                ("ms_total", ctypes.c_double)]


class BatchStats(ctypes.Structure):
    _fields_ = [("passes", ctypes.c_int32), ("tile_edges", ctypes.c_int32), ("blocks", ctypes.c_int32),
                ("max_link", ctypes.c_int32), ("total_edges", ctypes.c_int64),
                ("total_vertices", ctypes.c_int64), ("ms_total", ctypes.c_double), ("pass_ms", ctypes.c_float * 32),
                ("atomics", ctypes.c_int64), ("chase_reads", ctypes.c_int64), ("edges_read", ctypes.c_int64),
                ("survivors_written", ctypes.c_int64)]


class Peaks(ctypes.Structure):
    _fields_ = [("copy_gbps", ctypes.c_double), ("copy_bytes", ctypes.c_double), ("read_gbps", ctypes.c_double),
                ("table_bytes", ctypes.c_int64 * 3), ("gather_gps", ctypes.c_double * 3),
                ("atomic_gps", ctypes.c_double * 3), ("accesses", ctypes.c_double)]


_lib = None
_VP = ctypes.c_void_p


def lib():
    """Load libccmi.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built (run __graft_entry__.build()); no fallback exists")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "cc_version": (ctypes.c_int, []),
            "cc_last_error": (ctypes.c_char_p, []),
            "cc_default_options": (None, [ctypes.POINTER(Options)]),
            "cc_label": (ctypes.c_int, [_VP, _VP, ctypes.c_int64, ctypes.c_int32, _VP, _VP]),
            "cc_label_ex": (ctypes.c_int, [_VP, _VP, ctypes.c_int64, ctypes.c_int32, _VP, _VP,
                                           ctypes.POINTER(Options), ctypes.POINTER(Stats)]),
            "cc_label_batched": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_int32, _VP, _VP]),
            "cc_label_batched_ex": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_int32, _VP, _VP, ctypes.c_int32,
                                                   ctypes.c_int32, ctypes.POINTER(BatchStats)]),
            "cc_router_load": (ctypes.c_int, [ctypes.c_char_p]),
            "cc_router_set": (ctypes.c_int, [_VP]),
            "cc_router_loaded": (ctypes.c_int, []),
            "cc_degree": (ctypes.c_int, [_VP, _VP, ctypes.c_int64, ctypes.c_int32, _VP, _VP]),
            "cc_degree_histograms": (ctypes.c_int, [_VP, ctypes.c_int32, _VP, _VP, _VP, ctypes.c_int64,
                                                    ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                                                    _VP]),
            "cc_powerlaw_ks": (ctypes.c_int, [_VP, _VP, ctypes.c_int64, _VP]),
            "cc_csr": (ctypes.c_int, [_VP, _VP, ctypes.c_int64, ctypes.c_int32, _VP, _VP, _VP, _VP]),
            "cc_bfs": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, _VP,
                                      ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), _VP]),
            "cc_bfs_filter": (ctypes.c_int, [_VP, _VP, ctypes.c_int64, ctypes.c_int32, _VP, _VP, _VP, _VP,
                                             ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32), _VP]),
            "cc_mlp_forward": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, _VP, _VP]),
            "cc_mlp_sgd_step": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int32, ctypes.c_float, _VP,
                                               ctypes.POINTER(ctypes.c_float), _VP]),
            "cc_release_workspace": (ctypes.c_int, []),
            "cc_workspace_size": (ctypes.c_int64, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32]),
            "cc_shutdown": (ctypes.c_int, []),
            "cc_label_noalloc": (ctypes.c_int, [_VP, _VP, ctypes.c_int64, ctypes.c_int32, _VP, _VP]),
            "cc_check_labels": (ctypes.c_int, [_VP, _VP, ctypes.c_int64, ctypes.c_int32, _VP, _VP,
                                               ctypes.POINTER(ctypes.c_int64)]),
            "cc_debug_fail_alloc": (ctypes.c_int, [ctypes.c_int64]),
            "cc_measure_peaks": (ctypes.c_int, [ctypes.POINTER(Peaks), _VP]),
            "cc_label_tuples": (ctypes.c_int, [_VP, _VP, ctypes.c_int64, ctypes.c_int32, _VP, _VP, ctypes.c_int32,
                                               ctypes.POINTER(TupleStats)]),
            "cc_label64": (ctypes.c_int, [_VP, _VP, ctypes.c_int64, ctypes.c_int64, _VP, _VP,
                                          ctypes.POINTER(ctypes.c_int64), _VP]),
            "cc_label64_ex": (ctypes.c_int, [_VP, _VP, ctypes.c_int64, ctypes.c_int64, _VP, _VP,
                                             ctypes.POINTER(ctypes.c_int64), _VP, ctypes.POINTER(Options),
                                             ctypes.POINTER(Stats)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = L
        # release the library's device and pinned memory while the HIP
        # runtime is still up (Python's exit handlers run before the C ones)
        atexit.register(_shutdown_at_exit)
    return _lib


def _shutdown_at_exit():
    if _lib is not None:
        _lib.cc_shutdown()


def _check(rc: int):
    if rc != CC_OK:
        raise CCError(rc, lib().cc_last_error().decode(errors="replace"))


def _dev(t: torch.Tensor, dtype: torch.dtype, name: str):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return _VP(t.data_ptr() if t.numel() else 0)


def _stream():
    return _VP(torch.cuda.current_stream().cuda_stream)


def version() -> int:
    return lib().cc_version()


def label(u: torch.Tensor, v: torch.Tensor, n: int, route=None, out: torch.Tensor | None = None,
          stats: bool = False, max_passes: int = 0, tau: float = 0.05, theta: float = 8.0,
          profile: bool = False, workspace: torch.Tensor | None = None, scratch=None, check: bool = False):
    """labels[x] = min vertex id of x's component; (u[i], v[i]) are undirected edges.

    workspace: a uint8 device tensor of at least workspace_size(m, n, route)
    bytes used as the call's only device scratch; scratch: "cached" (default:
    the library's kept per-device workspace, calls serialise on it) or "pool"
    (stream-ordered allocations from the library's pool, no lock); check:
    the library's device-side invariant checks (cc_options.check)."""
    m = int(u.numel())
    if int(v.numel()) != m:
        raise ValueError("u and v differ in length")
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.int32, device=u.device if u.is_cuda else "cuda")
    opt = Options()
    lib().cc_default_options(ctypes.byref(opt))
    opt.route = _ROUTE_ARG[route] if not isinstance(route, int) else route
    opt.max_passes = max_passes
    opt.tau = tau
    opt.theta = theta
    opt.profile = 1 if profile else 0
    opt.scratch = _SCRATCH_ARG[scratch]
    opt.check = 1 if check else 0
    if workspace is not None:
        opt.workspace = _dev(workspace, torch.uint8, "workspace")
        opt.workspace_bytes = int(workspace.numel())
    st = Stats()
    rc = lib().cc_label_ex(_dev(u, torch.int32, "u"), _dev(v, torch.int32, "v"), m, n,
                           _dev(out, torch.int32, "labels"), _stream(), ctypes.byref(opt),
                           ctypes.byref(st) if stats else None)
    _check(rc)
    return (out, st.to_dict()) if stats else out


def check_labels(u: torch.Tensor, v: torch.Tensor, n: int, labels: torch.Tensor) -> dict:
    """Device check of a labelling (cc_check_labels): counts of edges whose
    ends differ in label (I1), vertices breaking I2, and out-of-range edges."""
    m = int(u.numel())
    if int(v.numel()) != m:
        raise ValueError("u and v differ in length")
    bad = (ctypes.c_int64 * 3)()
    _check(lib().cc_check_labels(_dev(u, torch.int32, "u"), _dev(v, torch.int32, "v"), m, n,
                                 _dev(labels, torch.int32, "labels"), _stream(), bad))
    return {"edges_split": int(bad[0]), "vertices_bad": int(bad[1]), "edges_out_of_range": int(bad[2])}


def measure_peaks() -> dict:
    """Measured ceilings of the current device (cc_measure_peaks): copy GB/s,
    and random gathers / returning atomicMin (G/s) on L2-, Infinity-Cache- and
    HBM-sized tables."""
    p = Peaks()
    _check(lib().cc_measure_peaks(ctypes.byref(p), _stream()))
    names = ("l2_2MiB", "mall_64MiB", "hbm_4GiB")
    return {"copy_GBps": round(p.copy_gbps, 1), "read_GBps": round(p.read_gbps, 1),
            "gather_Gps": {nm: round(p.gather_gps[k], 2) for k, nm in enumerate(names)},
            "atomicmin_Gps": {nm: round(p.atomic_gps[k], 2) for k, nm in enumerate(names)},
            "table_bytes": [int(x) for x in p.table_bytes], "accesses_per_launch": int(p.accesses)}


def debug_fail_alloc(nth: int) -> None:
    """Make the library's nth allocation from now fail (cc_debug_fail_alloc); 0 cancels."""
    _check(lib().cc_debug_fail_alloc(int(nth)))


def label_tuples(u: torch.Tensor, v: torch.Tensor, n: int, out: torch.Tensor | None = None, exclude: bool = False):
    """Algorithm 1 with radix sorts (cc_label_tuples): (labels, stats dict);
    exclude sets completed partitions aside (Section III-A.4)."""
    m = int(u.numel())
    if int(v.numel()) != m:
        raise ValueError("u and v differ in length")
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.int32, device=u.device)
    st = TupleStats()
    _check(lib().cc_label_tuples(_dev(u, torch.int32, "u"), _dev(v, torch.int32, "v"), m, n,
                                 _dev(out, torch.int32, "labels"), _stream(), 1 if exclude else 0, ctypes.byref(st)))
    return out, {k: getattr(st, k) for k, _ in TupleStats._fields_ if k != "reserved"}


def label64(u: torch.Tensor, v: torch.Tensor, n_max: int = 0, route=None, stats: bool = False):
    """Arbitrary 64-bit ids: (ids, labels) as int64 device tensors, each
    distinct endpoint id once (unspecified order) with the smallest id of its
    component (cc_label64)."""
    m = int(u.numel())
    if int(v.numel()) != m:
        raise ValueError("u and v differ in length")
    cap = int(n_max) if n_max > 0 else 2 * m
    ids = torch.empty(max(cap, 1), dtype=torch.int64, device=u.device)
    labels = torch.empty(max(cap, 1), dtype=torch.int64, device=u.device)
    n = ctypes.c_int64(0)
    opt = Options()
    lib().cc_default_options(ctypes.byref(opt))
    opt.route = _ROUTE_ARG[route] if not isinstance(route, int) else route
    st = Stats()
    _check(lib().cc_label64_ex(_dev(u, torch.int64, "u"), _dev(v, torch.int64, "v"), m, int(n_max),
                               _dev(ids, torch.int64, "ids"), _dev(labels, torch.int64, "labels"),
                               ctypes.byref(n), _stream(), ctypes.byref(opt), ctypes.byref(st) if stats else None))
    k = int(n.value)
    return (ids[:k], labels[:k], st.to_dict()) if stats else (ids[:k], labels[:k])


NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024


def label_noalloc(u: torch.Tensor, v: torch.Tensor, n: int, out: torch.Tensor):
    """cc_label_noalloc: plain SV labels with no allocation (scratch is the
    library's fixed per-GPU array; out must be given)."""
    m = int(u.numel())
    if int(v.numel()) != m:
        raise ValueError("u and v differ in length")
    _check(lib().cc_label_noalloc(_dev(u, torch.int32, "u"), _dev(v, torch.int32, "v"), m, n,
                                  _dev(out, torch.int32, "labels"), _stream()))
    return out


def label_batched(u, v, edge_off, vert_off, out=None, tile_edges: int = 0, max_link: int = 0,
                  stats: bool = False):
    """Graph-local labels of G graphs (see cc_label_batched); 0 = autotuned launch shape."""
    G = int(edge_off.numel()) - 1
    if out is None:
        total = int(vert_off[-1].item()) if G >= 0 else 0
        out = torch.empty(max(total, 0), dtype=torch.int32, device=u.device)
    st = BatchStats()
    rc = lib().cc_label_batched_ex(_dev(u, torch.int32, "u"), _dev(v, torch.int32, "v"),
                                   _dev(edge_off, torch.int64, "edge_off"), _dev(vert_off, torch.int64, "vert_off"),
                                   G, _dev(out, torch.int32, "labels"), _stream(), tile_edges, max_link,
                                   ctypes.byref(st) if stats else None)
    _check(rc)
    if stats:
        d = {k: getattr(st, k) for k, _ in BatchStats._fields_ if k != "pass_ms"}
        d["pass_ms"] = [round(float(x), 4) for x in st.pass_ms][: st.passes + 1]
        return out, d
    return out


def degree(u, v, n):
    out = torch.empty(n, dtype=torch.int32, device=u.device)
    _check(lib().cc_degree(_dev(u, torch.int32, "u"), _dev(v, torch.int32, "v"), int(u.numel()), n,
                           _dev(out, torch.int32, "deg"), _stream()))
    return out


def degree_histograms(deg: torch.Tensor, tail_cap: int | None = None):
    n = int(deg.numel())
    if tail_cap is None:
        tail_cap = max(1, n)
    hist64 = torch.empty(64, dtype=torch.int64, device=deg.device)
    histx = torch.empty(4096, dtype=torch.int64, device=deg.device)
    tail = torch.empty(max(tail_cap, 1), dtype=torch.int32, device=deg.device)
    cnt = ctypes.c_int64(0)
    amax = ctypes.c_int32(-1)
    _check(lib().cc_degree_histograms(_dev(deg, torch.int32, "deg"), n, _dev(hist64, torch.int64, "hist64"),
                                      _dev(histx, torch.int64, "histx"), _dev(tail, torch.int32, "tail"), tail_cap,
                                      ctypes.byref(cnt), ctypes.byref(amax), _stream()))
    k = min(int(cnt.value), tail_cap)
    return hist64, histx, tail[:k], int(cnt.value), int(amax.value)


def powerlaw_ks(histx, tail):
    """Host fit: histx int64[4096], tail int32 (numpy arrays)."""
    import numpy as np
    hx = np.ascontiguousarray(np.asarray(histx, dtype=np.int64))
    tl = np.ascontiguousarray(np.asarray(tail, dtype=np.int32))
    out = (ctypes.c_double * 5)()
    _check(lib().cc_powerlaw_ks(_VP(hx.ctypes.data), _VP(tl.ctypes.data if tl.size else 0), int(tl.size), out))
    return dict(ks=out[0], alpha=out[1], dmin=int(out[2]), ntail=int(out[3]), candidates=int(out[4]))


def csr(u, v, n):
    """(off int64[n+1], adj int32[2m], deg int32[n]) of the undirected graph."""
    m = int(u.numel())
    off = torch.empty(n + 1, dtype=torch.int64, device=u.device)
    adj = torch.empty(max(2 * m, 1), dtype=torch.int32, device=u.device)
    deg = torch.empty(max(n, 1), dtype=torch.int32, device=u.device)
    _check(lib().cc_csr(_dev(u, torch.int32, "u"), _dev(v, torch.int32, "v"), m, n, _dev(deg, torch.int32, "deg"),
                        _dev(off, torch.int64, "off"), _dev(adj, torch.int32, "adj"), _stream()))
    return off, adj[: 2 * m], deg[:n]


def bfs(off, adj, n, seed):
    words = (n + 31) // 32
    vis = torch.empty(max(words, 1), dtype=torch.int32, device=off.device)
    lv = ctypes.c_int32(0)
    bu = ctypes.c_int32(0)
    _check(lib().cc_bfs(_dev(off, torch.int64, "off"), _dev(adj, torch.int32, "adj"), n, int(adj.numel()), seed,
                        _dev(vis, torch.int32, "visited"), ctypes.byref(lv), ctypes.byref(bu), _stream()))
    return vis[:words], int(lv.value), int(bu.value)


def bfs_filter(u, v, n, visited):
    m = int(u.numel())
    labels = torch.empty(n, dtype=torch.int32, device=u.device)
    fu = torch.empty(max(m, 1), dtype=torch.int32, device=u.device)
    fv = torch.empty(max(m, 1), dtype=torch.int32, device=u.device)
    kept = ctypes.c_int64(0)
    lab = ctypes.c_int32(-1)
    _check(lib().cc_bfs_filter(_dev(u, torch.int32, "u"), _dev(v, torch.int32, "v"), m, n,
                               _dev(visited, torch.int32, "visited"), _dev(labels, torch.int32, "labels"),
                               _dev(fu, torch.int32, "fu"), _dev(fv, torch.int32, "fv"), ctypes.byref(kept),
                               ctypes.byref(lab), _stream()))
    k = int(kept.value)
    return labels, fu[:k], fv[:k], int(lab.value)


def mlp_forward(params, x):
    B = int(x.shape[0])
    out = torch.empty((B, 3), dtype=torch.float32, device=x.device)
    _check(lib().cc_mlp_forward(_dev(params, torch.float32, "params"), _dev(x, torch.float32, "x"), B,
                                _dev(out, torch.float32, "logits"), _stream()))
    return out


def mlp_sgd_step(params, x, y, lr, want_grads=False):
    B = int(x.shape[0])
    grads = torch.empty(ROUTER_NPARAMS, dtype=torch.float32, device=x.device) if want_grads else None
    loss = ctypes.c_float(0.0)
    _check(lib().cc_mlp_sgd_step(_dev(params, torch.float32, "params"), _dev(x, torch.float32, "x"),
                                 _dev(y, torch.int32, "y"), B, float(lr),
                                 _dev(grads, torch.float32, "grads") if grads is not None else None,
                                 ctypes.byref(loss), _stream()))
    return float(loss.value), grads


def router_load(path: str):
    _check(lib().cc_router_load(path.encode()))


def router_set(params_host) -> None:
    import numpy as np
    if params_host is None:
        _check(lib().cc_router_set(None))
        return
    p = np.ascontiguousarray(np.asarray(params_host, dtype=np.float32))
    if p.size != ROUTER_NPARAMS:
        raise ValueError("router parameter count")
    _check(lib().cc_router_set(_VP(p.ctypes.data)))


def router_loaded() -> bool:
    return bool(lib().cc_router_loaded())


def workspace_size(m: int, n: int, route=None) -> int:
    """Bytes of device scratch a label() call on m edges and n vertices may use."""
    r = lib().cc_workspace_size(int(m), int(n), _ROUTE_ARG[route] if not isinstance(route, int) else route)
    if r < 0:
        _check(int(r))
    return int(r)


def release_workspace():
    _check(lib().cc_release_workspace())


def shutdown():
    """Free everything the library holds (no call may be running)."""
    _check(lib().cc_shutdown())

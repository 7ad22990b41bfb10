"""Python binding of the HDD C ABI (include/hdd.h).

Argument marshalling only: every step of the computation runs in the HIP
library libhdd.so built in-tree.  PyTorch provides device memory (the
workspace, device inputs/outputs) and streams.  Importing this module fails
loudly if the library is missing; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhdd.so")

HDD_OK = 0
HDD_EINVAL = -1
HDD_ENOMEM = -2
HDD_ENOTSPD = -3
HDD_ENOTCONVERGED = -4
HDD_EDEVICE = -5
HDD_ESTATE = -6
HDD_FP64 = 0
HDD_FP32_REFINE = 1
HDD_MEM_HOST = 0
HDD_MEM_DEVICE = 1
HDD_FLAG_NO_MFMA = 1
HDD_FLAG_KEEP_DIRICHLET = 2
HDD_FLAG_BLOCK8 = 4
HDD_FLAG_KEEP_FRAMES = 8
HDD_FLAG_NO_GRAPH = 16
HDD_FLAG_LOWRANK = 32
HDD_FLAG_NO_FUSED = 64

EXPORTED = [
    "hdd_default_opts", "hdd_workspace_size", "hdd_create", "hdd_build", "hdd_query_points",
    "hdd_query_interface", "hdd_query_mean", "hdd_query_node_means", "hdd_loglik", "hdd_solve_full", "hdd_solve_rhs", "hdd_solve_rhs_coarse", "hdd_get_solution_coarse", "hdd_get_solution",
    "hdd_error_estimate", "hdd_sync", "hdd_last_node", "hdd_destroy", "hdd_strerror",
    "hdd_plan_summary", "hdd_plan_node", "hdd_plan_level", "hdd_debug_node_schur",
    "hdd_timing_enable", "hdd_timing_get", "hdd_mfma_selftest", "hdd_debug_frame",
    "hdd_timing_get_level", "hdd_query_points_ragged", "hdd_loglik_ragged",
    "hdd_server_create", "hdd_server_slots", "hdd_server_submit", "hdd_server_poll", "hdd_server_result",
    "hdd_server_stats", "hdd_server_destroy", "hdd_sample_status", "hdd_create_static", "hdd_autotune", "hdd_graph_info", "hdd_server_memory", "hdd_lowrank_info", "hdd_query_skeleton",
]
MAX_QUERY_POINTS = 4096
STATIC_WORKSPACE_BYTES = 64 << 20

SERVER_MAX_MESHES = 8
SERVER_MAX_POINTS = 256


class HddOpts(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("leaf", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("fp64_top_levels", ctypes.c_int32), ("max_refine", ctypes.c_int32), ("flags", ctypes.c_int32),
        ("refine_tol", ctypes.c_double), ("reserved", ctypes.c_int32 * 8),
    ]


class ServerOpts(ctypes.Structure):
    _fields_ = [
        ("n_meshes", ctypes.c_int32), ("n", ctypes.c_int32 * SERVER_MAX_MESHES),
        ("leaf", ctypes.c_int32 * SERVER_MAX_MESHES), ("precision", ctypes.c_int32), ("slots", ctypes.c_int32),
        ("hbm_budget", ctypes.c_double), ("max_refine", ctypes.c_int32), ("reserved", ctypes.c_int32 * 7),
    ]


class HddError(RuntimeError):
    def __init__(self, code: int, where: str, node: int = 0):
        self.code = code
        self.node = node
        extra = f", first failing node {node - 1}" if node else ""
        super().__init__(f"{where}: {strerror(code)} ({code}{extra})")


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HDD HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    popts = ctypes.POINTER(HddOpts)
    sig = {
        "hdd_default_opts": [i32, i32, popts],
        "hdd_workspace_size": [popts, i32, ctypes.POINTER(ctypes.c_size_t)],
        "hdd_create": [popts, i32, P, P, ctypes.c_size_t, ctypes.POINTER(P)],
        "hdd_create_static": [popts, i32, P, ctypes.POINTER(P)],
        "hdd_autotune": [P, i32, P],
        "hdd_graph_info": [P, P],
        "hdd_lowrank_info": [P, P],
        "hdd_query_skeleton": [P, i32, P, ctypes.POINTER(i32), i32],
        "hdd_build": [P, i32, P, P, P, i32],
        "hdd_query_points": [P, i32, P, P, i32],
        "hdd_query_interface": [P, i32, i32, P, ctypes.POINTER(i32), i32],
        "hdd_sample_status": [P, P],
        "hdd_query_mean": [P, P, P, i32],
        "hdd_query_node_means": [P, P, i32],
        "hdd_solve_rhs": [P, P, P, i32],
        "hdd_solve_rhs_coarse": [P, P, P, i32],
        "hdd_get_solution_coarse": [P, i32, P, i32],
        "hdd_loglik": [P, i32, P, P, dbl, i32, P, i32],
        "hdd_solve_full": [P],
        "hdd_get_solution": [P, i32, P, i32],
        "hdd_error_estimate": [P, P, ctypes.POINTER(i32)],
        "hdd_sync": [P],
        "hdd_last_node": [P],
        "hdd_destroy": [P],
        "hdd_strerror": [ctypes.c_int],
        "hdd_plan_summary": [popts, P],
        "hdd_plan_node": [popts, i32, i32, P, P],
        "hdd_plan_level": [popts, i32, P],
        "hdd_debug_node_schur": [P, i32, i32, i32, P, P],
        "hdd_timing_enable": [P, i32],
        "hdd_timing_get": [P, i32, ctypes.POINTER(dbl), ctypes.POINTER(i64), ctypes.POINTER(dbl)],
        "hdd_mfma_selftest": [i32, P],
        "hdd_debug_frame": [P, i32, i32, i32, P, ctypes.POINTER(i32)],
        "hdd_timing_get_level": [P, i32, i32, ctypes.POINTER(dbl), ctypes.POINTER(i64), ctypes.POINTER(dbl),
                                 ctypes.POINTER(dbl)],
        "hdd_query_points_ragged": [P, P, P, P, i32],
        "hdd_loglik_ragged": [P, P, P, P, P, i32, P, i32],
        "hdd_server_create": [ctypes.POINTER(ServerOpts), P, ctypes.POINTER(P)],
        "hdd_server_slots": [P, ctypes.POINTER(i32)],
        "hdd_server_submit": [P, i32, P, i32, P, P, dbl, ctypes.POINTER(i64)],
        "hdd_server_poll": [P, i64, ctypes.POINTER(i32)],
        "hdd_server_result": [P, i64, P, ctypes.POINTER(dbl), P],
        "hdd_server_stats": [P, P],
        "hdd_server_memory": [P, P],
        "hdd_server_destroy": [P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p if name == "hdd_strerror" else ctypes.c_int
    return lib


_lib = _load()


def strerror(code: int) -> str:
    return _lib.hdd_strerror(int(code)).decode()


def _check(code: int, where: str):
    if code != HDD_OK:
        raise HddError(code, where)


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def hdd_default_opts(n: int, precision: int = HDD_FP64, **overrides) -> HddOpts:
    o = HddOpts()
    _check(_lib.hdd_default_opts(int(n), int(precision), ctypes.byref(o)), "hdd_default_opts")
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def hdd_workspace_size(opts: HddOpts, max_samples: int) -> int:
    b = ctypes.c_size_t(0)
    _check(_lib.hdd_workspace_size(ctypes.byref(opts), int(max_samples), ctypes.byref(b)), "hdd_workspace_size")
    return b.value


def hdd_plan_summary(opts: HddOpts) -> dict:
    out = np.zeros(6, dtype=np.int64)
    _check(_lib.hdd_plan_summary(ctypes.byref(opts), _np_ptr(out)), "hdd_plan_summary")
    keys = ["levels", "nodes", "depth_leaf", "depth_block", "frame_elems", "flops"]
    return dict(zip(keys, (int(v) for v in out)))


def hdd_plan_node(opts: HddOpts, depth: int, index: int):
    info = np.zeros(6, dtype=np.int32)
    _check(_lib.hdd_plan_node(ctypes.byref(opts), int(depth), int(index), _np_ptr(info), None), "hdd_plan_node")
    ids = np.zeros(int(info[4] + info[5]), dtype=np.int32)
    _check(_lib.hdd_plan_node(ctypes.byref(opts), int(depth), int(index), _np_ptr(info), _np_ptr(ids)),
           "hdd_plan_node")
    return dict(x0=int(info[0]), y0=int(info[1]), w=int(info[2]), h=int(info[3]),
                gam=int(info[4]), bnd=int(info[5]), ids=ids)


def hdd_plan_level(opts: HddOpts, depth: int) -> dict:
    out = np.zeros(4, dtype=np.int32)
    _check(_lib.hdd_plan_level(ctypes.byref(opts), int(depth), _np_ptr(out)), "hdd_plan_level")
    return dict(nodes=int(out[0]), gam=int(out[1]), max_U=int(out[2]), fp64=bool(out[3]))


def hdd_mfma_selftest(dtype: int) -> np.ndarray:
    n = 32 if dtype == 0 else 16
    out = np.zeros(n * n)
    _check(_lib.hdd_mfma_selftest(int(dtype), _np_ptr(out)), "hdd_mfma_selftest")
    return out.reshape(n, n)


def _is_torch_cuda(x) -> bool:
    return hasattr(x, "is_cuda") and bool(x.is_cuda)


def _ptr(x):
    """(pointer, mem kind) of a numpy array or a torch CUDA tensor."""
    if _is_torch_cuda(x):
        assert x.is_contiguous()
        return ctypes.c_void_p(x.data_ptr()), HDD_MEM_DEVICE
    return _np_ptr(x), HDD_MEM_HOST


def _ragged(xy_per_sample, n_samples: int):
    assert len(xy_per_sample) == n_samples
    parts = [np.asarray(a, dtype=np.float64).reshape(-1, 2) for a in xy_per_sample]
    off = np.zeros(n_samples + 1, dtype=np.int32)
    off[1:] = np.cumsum([len(p) for p in parts])
    return off, np.ascontiguousarray(np.concatenate(parts))


class HDD:
    """One handle: a planned tree with device memory for up to max_samples samples."""

    def __init__(self, opts: HddOpts, max_samples: int, stream=None, workspace: str = "torch"):
        """workspace: "torch" (a torch device buffer passed to hdd_create),
        "library" (hdd_create allocates it) or "static" (hdd_create_static:
        the library's static device array, no allocation)."""
        import torch

        self.opts = opts
        self.n = opts.n
        self.nc = opts.n + 1
        self.max_samples = int(max_samples)
        self.n_samples = 0
        self._ws = None
        wptr, wbytes = None, 0
        if workspace == "torch":
            wbytes = hdd_workspace_size(opts, max_samples)
            self._ws = torch.empty(wbytes, dtype=torch.uint8, device="cuda")
            wptr = ctypes.c_void_p(self._ws.data_ptr())
        sptr = None
        if stream is not None:
            sptr = ctypes.c_void_p(stream.cuda_stream)
        self.stream = stream
        h = ctypes.c_void_p()
        if workspace == "static":
            _check(_lib.hdd_create_static(ctypes.byref(opts), self.max_samples, sptr, ctypes.byref(h)),
                   "hdd_create_static")
        else:
            _check(_lib.hdd_create(ctypes.byref(opts), self.max_samples, sptr, wptr, ctypes.c_size_t(wbytes),
                                   ctypes.byref(h)), "hdd_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            _lib.hdd_destroy(self.h)
            self.h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- Leaves to Root -----------------------------------------------------
    def build(self, kappa, f):
        if not _is_torch_cuda(kappa):
            kappa = np.ascontiguousarray(kappa, dtype=np.float64)
            f = np.ascontiguousarray(f, dtype=np.float64)
        ns = int(kappa.shape[0])
        assert tuple(kappa.shape[1:]) == (self.nc, self.nc, 2) and tuple(f.shape) == (self.nc + 1, self.nc + 1)
        kp, mem = _ptr(kappa)
        fp, mem2 = _ptr(f)
        assert mem == mem2
        self._keep = (kappa, f)
        _check(_lib.hdd_build(self.h, ns, kp, fp, None, mem), "hdd_build")
        self.n_samples = ns

    # -- queries ----------------------------------------------------------------
    def query_points(self, xy, out=None) -> np.ndarray:
        xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
        if out is None:
            res = np.zeros((self.n_samples, len(xy)))
            _check(_lib.hdd_query_points(self.h, len(xy), _np_ptr(xy), _np_ptr(res), HDD_MEM_HOST),
                   "hdd_query_points")
            return res
        op, mem = _ptr(out)
        _check(_lib.hdd_query_points(self.h, len(xy), _np_ptr(xy), op, mem), "hdd_query_points")
        return out

    def query_interface(self, depth: int = 0, index: int = 0, out=None) -> np.ndarray:
        """u on the interface gamma of tree node (depth, index), [n_samples][|gamma|],
        entries in the order of hdd_plan_node's ids; (0, 0) is the root midline."""
        ln = ctypes.c_int32(0)
        if out is None:
            # |gamma| is uniform on a level; hdd_plan_level plans the tree on
            # the host, so it is asked once per depth and handle
            cache = self.__dict__.setdefault("_gam", {})
            if depth not in cache:
                cache[depth] = hdd_plan_level(self.opts, depth)["gam"]
            g = cache[depth]
            res = np.zeros((self.n_samples, g))
            _check(_lib.hdd_query_interface(self.h, int(depth), int(index), _np_ptr(res), ctypes.byref(ln),
                                            HDD_MEM_HOST), "hdd_query_interface")
            assert ln.value == g
            return res
        op, mem = _ptr(out)
        _check(_lib.hdd_query_interface(self.h, int(depth), int(index), op, ctypes.byref(ln), mem),
               "hdd_query_interface")
        return out

    def query_skeleton(self, depth: int, out=None):
        """u on every interface of the nodes above `depth` (plan order),
        [n_samples][len]; in float64 without the full field only those
        interfaces are solved."""
        ln = ctypes.c_int32(0)
        if out is None:
            if getattr(self, "_levels", None) is None:  # planning the tree once per handle
                self._levels = [hdd_plan_level(self.opts, d) for d in range(hdd_plan_summary(self.opts)["levels"])]
            total = sum(lv["nodes"] * lv["gam"] for lv in self._levels[:depth])
            res = np.zeros((self.n_samples, total))
            _check(_lib.hdd_query_skeleton(self.h, int(depth), _np_ptr(res), ctypes.byref(ln), HDD_MEM_HOST),
                   "hdd_query_skeleton")
            assert ln.value == total
            return res
        op, mem = _ptr(out)
        _check(_lib.hdd_query_skeleton(self.h, int(depth), op, ctypes.byref(ln), mem), "hdd_query_skeleton")
        return out

    def sample_status(self) -> np.ndarray:
        """Per-sample status codes (HDD_OK, HDD_EINVAL, HDD_ENOTSPD, HDD_ENOTCONVERGED)."""
        st = np.zeros(max(self.n_samples, 1), dtype=np.int32)
        _check(_lib.hdd_sample_status(self.h, _np_ptr(st)), "hdd_sample_status")
        return st[: self.n_samples]

    def query_mean(self, rect: Sequence[float]) -> np.ndarray:
        r = np.ascontiguousarray(rect, dtype=np.float64)
        res = np.zeros(self.n_samples)
        _check(_lib.hdd_query_mean(self.h, _np_ptr(r), _np_ptr(res), HDD_MEM_HOST), "hdd_query_mean")
        return res

    def query_node_means(self, out=None) -> np.ndarray:
        """Mean of u over every node of the tree down to the blocks,
        [n_samples][nodes] in plan order (root, then depth by depth)."""
        if out is None:
            nodes = hdd_plan_summary(self.opts)["nodes"]
            res = np.zeros((self.n_samples, nodes))
            _check(_lib.hdd_query_node_means(self.h, _np_ptr(res), HDD_MEM_HOST), "hdd_query_node_means")
            return res
        op, mem = _ptr(out)
        _check(_lib.hdd_query_node_means(self.h, op, mem), "hdd_query_node_means")
        return out

    def loglik(self, xy, y, sigma: float, normalized: bool = False, out=None):
        xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
        if out is None:
            y = np.ascontiguousarray(y, dtype=np.float64)
            res = np.zeros(self.n_samples)
            _check(_lib.hdd_loglik(self.h, len(xy), _np_ptr(xy), _np_ptr(y), float(sigma), int(normalized),
                                   _np_ptr(res), HDD_MEM_HOST), "hdd_loglik")
            return res
        yp, mem = _ptr(y)
        op, mem2 = _ptr(out)
        assert mem == mem2 == HDD_MEM_DEVICE
        _check(_lib.hdd_loglik(self.h, len(xy), _np_ptr(xy), yp, float(sigma), int(normalized), op, mem),
               "hdd_loglik")
        return out

    def query_points_ragged(self, xy_per_sample):
        """Values at sample-specific sites: xy_per_sample[s] is an [n_s, 2]
        array for sample s; returns a list of arrays."""
        off, xy = _ragged(xy_per_sample, self.n_samples)
        res = np.zeros(int(off[-1]))
        _check(_lib.hdd_query_points_ragged(self.h, _np_ptr(off), _np_ptr(xy), _np_ptr(res), HDD_MEM_HOST),
               "hdd_query_points_ragged")
        return [res[off[s]:off[s + 1]] for s in range(self.n_samples)]

    def loglik_ragged(self, xy_per_sample, y_per_sample, sigma, normalized: bool = False):
        off, xy = _ragged(xy_per_sample, self.n_samples)
        y = np.ascontiguousarray(np.concatenate([np.asarray(v, dtype=np.float64).ravel() for v in y_per_sample]))
        assert len(y) == off[-1]
        sg = np.ascontiguousarray(np.broadcast_to(np.asarray(sigma, dtype=np.float64), (self.n_samples,)))
        res = np.zeros(self.n_samples)
        _check(_lib.hdd_loglik_ragged(self.h, _np_ptr(off), _np_ptr(xy), _np_ptr(y), _np_ptr(sg), int(normalized),
                                      _np_ptr(res), HDD_MEM_HOST), "hdd_loglik_ragged")
        return res

    def solve_full(self, check: bool = True) -> int:
        code = _lib.hdd_solve_full(self.h)
        if check:
            _check(code, "hdd_solve_full")
        return code

    def solve_rhs(self, f, g=None, check: bool = True, coarse: bool = False) -> int:
        """Field for another load f (and Dirichlet data g, nodal [N+2][N+2])
        on the built operators; numpy arrays or CUDA tensors.  coarse: f is
        nodal on the mesh of twice the step, [Nc/2+1]^2."""
        if _is_torch_cuda(f):
            fp, mem = _ptr(f)
            gp = _ptr(g)[0] if g is not None else None
        else:
            f = np.ascontiguousarray(f, dtype=np.float64)
            fp, mem = _np_ptr(f), HDD_MEM_HOST
            if g is not None:
                g = np.ascontiguousarray(g, dtype=np.float64)
            gp = _np_ptr(g) if g is not None else None
        fshape = (self.nc // 2 + 1,) * 2 if coarse else (self.nc + 1,) * 2
        assert tuple(f.shape) == fshape and (g is None or tuple(g.shape) == (self.nc + 1, self.nc + 1))
        self._keep_rhs = (f, g)
        fn = _lib.hdd_solve_rhs_coarse if coarse else _lib.hdd_solve_rhs
        code = fn(self.h, fp, gp, mem)
        if check:
            _check(code, "hdd_solve_rhs_coarse" if coarse else "hdd_solve_rhs")
        return code

    def solution_coarse(self, sample: int) -> np.ndarray:
        m1 = self.nc // 2 + 1
        u = np.zeros((m1, m1))
        _check(_lib.hdd_get_solution_coarse(self.h, int(sample), _np_ptr(u), HDD_MEM_HOST), "hdd_get_solution_coarse")
        return u

    def solution(self, sample: int) -> np.ndarray:
        u = np.zeros((self.nc + 1, self.nc + 1))
        _check(_lib.hdd_get_solution(self.h, int(sample), _np_ptr(u), HDD_MEM_HOST), "hdd_get_solution")
        return u

    def error_estimate(self):
        est = np.zeros(max(self.n_samples, 1))
        sw = ctypes.c_int32(0)
        _check(_lib.hdd_error_estimate(self.h, _np_ptr(est), ctypes.byref(sw)), "hdd_error_estimate")
        return est[: self.n_samples], sw.value

    def sync(self) -> int:
        return _lib.hdd_sync(self.h)

    def autotune(self, reps: int = 1) -> np.ndarray:
        """Per-level Schur-update tile chosen by timing (64, 128, or 0: no choice)."""
        levels = hdd_plan_summary(self.opts)["levels"]
        ch = np.zeros(levels, dtype=np.int32)
        _check(_lib.hdd_autotune(self.h, int(reps), _np_ptr(ch)), "hdd_autotune")
        return ch

    def lowrank_info(self) -> dict:
        out = np.zeros(6)
        _check(_lib.hdd_lowrank_info(self.h, _np_ptr(out)), "hdd_lowrank_info")
        return dict(dense_bytes=out[0], store_bytes=out[1], rank_bytes=out[2], lowrank_blocks=int(out[3]),
                    dense_blocks=int(out[4]), mean_rank=out[5])

    def graph_info(self) -> dict:
        out = np.zeros(4, dtype=np.int64)
        _check(_lib.hdd_graph_info(self.h, _np_ptr(out)), "hdd_graph_info")
        return dict(build_nodes=int(out[0]), solve_nodes=int(out[1]), sweep_nodes=int(out[2]),
                    launches=int(out[3]))

    def last_node(self) -> int:
        return _lib.hdd_last_node(self.h)

    def node_schur(self, sample: int, depth: int, index: int):
        info = hdd_plan_node(self.opts, depth, index)
        G = info["bnd"]
        S = np.zeros((G + 1, G + 1))
        ids = np.zeros(G, dtype=np.int32)
        _check(_lib.hdd_debug_node_schur(self.h, int(sample), int(depth), int(index), _np_ptr(S), _np_ptr(ids)),
               "hdd_debug_node_schur")
        return S[:G, :G], S[G, :G], ids

    def frame(self, sample: int, depth: int, index: int) -> np.ndarray:
        mx = hdd_plan_level(self.opts, depth)["max_U"] + 1
        out = np.zeros(mx * mx)
        U = ctypes.c_int32(0)
        _check(_lib.hdd_debug_frame(self.h, int(sample), int(depth), int(index), _np_ptr(out), ctypes.byref(U)),
               "hdd_debug_frame")
        n = U.value + 1
        return out[: n * n].reshape(n, n)

    # -- timing -------------------------------------------------------------------
    def timing_enable(self, mask: int):
        _check(_lib.hdd_timing_enable(self.h, int(mask)), "hdd_timing_enable")

    def timing_get(self, kind: int, level: int = -1, with_bytes: bool = False):
        """(ms, launches, flops[, bytes]) of the timed launches of `kind`."""
        ms = ctypes.c_double(0)
        n = ctypes.c_int64(0)
        fl = ctypes.c_double(0)
        by = ctypes.c_double(0)
        _check(_lib.hdd_timing_get_level(self.h, int(kind), int(level), ctypes.byref(ms), ctypes.byref(n),
                                         ctypes.byref(fl), ctypes.byref(by)), "hdd_timing_get_level")
        if with_bytes:
            return ms.value, n.value, fl.value, by.value
        return ms.value, n.value, fl.value


class Server:
    """Continuous-batching likelihood server (hdd_server_* in include/hdd.h):
    one HDD handle, stream and worker thread per mesh size."""

    def __init__(self, meshes, precision: int = HDD_FP32_REFINE, slots: int = 0, hbm_budget: float = 0.0,
                 leaves=None, f=None, max_refine: int = 0):
        o = ServerOpts()
        o.n_meshes = len(meshes)
        for i, n in enumerate(meshes):
            o.n[i] = int(n)
            o.leaf[i] = int(leaves[i]) if leaves else 0
        o.precision = int(precision)
        o.slots = int(slots)
        o.hbm_budget = float(hbm_budget)
        o.max_refine = int(max_refine)
        self.meshes = list(meshes)
        self._f = None
        fp = None
        if f is not None:
            self._f = [np.ascontiguousarray(a, dtype=np.float64) for a in f]
            arr = (ctypes.c_void_p * len(self._f))(*[a.ctypes.data for a in self._f])
            fp = ctypes.cast(arr, ctypes.c_void_p)
        h = ctypes.c_void_p()
        _check(_lib.hdd_server_create(ctypes.byref(o), fp, ctypes.byref(h)), "hdd_server_create")
        self.h = h
        sl = ctypes.c_int32(0)
        _check(_lib.hdd_server_slots(self.h, ctypes.byref(sl)), "hdd_server_slots")
        self.slots = sl.value

    def submit(self, mesh: int, kappa, xy, y=None, sigma: float = 1.0) -> int:
        kappa = np.ascontiguousarray(kappa, dtype=np.float64)
        xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
        yp = None
        if y is not None:
            y = np.ascontiguousarray(y, dtype=np.float64)
            yp = _np_ptr(y)
        rid = ctypes.c_int64(0)
        _check(_lib.hdd_server_submit(self.h, int(mesh), _np_ptr(kappa), len(xy), _np_ptr(xy), yp, float(sigma),
                                      ctypes.byref(rid)), "hdd_server_submit")
        return rid.value

    def poll(self, rid: int) -> bool:
        d = ctypes.c_int32(0)
        _check(_lib.hdd_server_poll(self.h, int(rid), ctypes.byref(d)), "hdd_server_poll")
        return bool(d.value)

    def result(self, rid: int, n_pts: int, with_status: bool = False):
        """(values [n_pts], loglik, times [queue, batch, total seconds, batch size]);
        with_status: the request's status code is returned as a fourth item
        instead of raising on a non-OK code."""
        vals = np.zeros(n_pts)
        ll = ctypes.c_double(0)
        times = np.zeros(4)
        code = _lib.hdd_server_result(self.h, int(rid), _np_ptr(vals), ctypes.byref(ll), _np_ptr(times))
        if with_status:
            return vals, ll.value, times, code
        _check(code, "hdd_server_result")
        return vals, ll.value, times

    def stats(self):
        out = np.zeros(4, dtype=np.int64)
        _check(_lib.hdd_server_stats(self.h, _np_ptr(out)), "hdd_server_stats")
        return dict(submitted=int(out[0]), completed=int(out[1]), batches=int(out[2]), queued=int(out[3]))

    def memory(self):
        out = np.zeros(4, dtype=np.int64)
        _check(_lib.hdd_server_memory(self.h, _np_ptr(out)), "hdd_server_memory")
        return dict(bytes=int(out[0]), resident=int(out[1]), evictions=int(out[2]), creations=int(out[3]))

    def close(self):
        if getattr(self, "h", None):
            _lib.hdd_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

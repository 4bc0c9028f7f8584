"""Thin ctypes binding of libocck (include/occk.h).  Argument marshalling only:
every step of the far-field exchange runs in the library's HIP kernels.
PyTorch provides device memory and streams."""
from __future__ import annotations

import ctypes as ct
import math
import os
from dataclasses import dataclass

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libocck.so")

OK, EINVAL, ENOMEM, EHIP, EHANDLE, ENONFINITE, ESTATE = 0, -1, -2, -3, -4, -5, -6
PREC_FP64, PREC_FP32, PREC_BF16X3, PREC_BF16X6 = 0, 1, 2, 3
RANK_FIXED, RANK_LEARNED = 0, 1
MAX_LEVELS = 13


class OcckError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"occk error {code}: {msg}")
        self.code = code


class _System(ct.Structure):
    _fields_ = [("natoms", ct.c_int32), ("xyz", ct.POINTER(ct.c_double)),
                ("nshell", ct.c_int32), ("shell_atom", ct.POINTER(ct.c_int32)),
                ("shell_l", ct.POINTER(ct.c_int32)), ("shell_exp", ct.POINTER(ct.c_double))]


class _Params(ct.Structure):
    _fields_ = [("split_mask", ct.c_int32), ("depth", ct.c_int32), ("ws", ct.c_int32),
                ("lmax", ct.c_int32), ("pair_log_thresh", ct.c_double), ("near_rule", ct.c_int32),
                ("ext_ws", ct.c_double), ("ext_tau", ct.c_double)]


class _Info(ct.Structure):
    _fields_ = [("nbasis", ct.c_int32), ("lmax", ct.c_int32), ("ncomp", ct.c_int32),
                ("depth", ct.c_int32), ("lmin", ct.c_int32), ("nleaf", ct.c_int32),
                ("nbox", ct.c_int32), ("boxes_per_level", ct.c_int32 * MAX_LEVELS),
                ("il_per_level", ct.c_int32 * MAX_LEVELS), ("n_il", ct.c_int64),
                ("n_edges", ct.c_int64), ("npairs", ct.c_int64), ("sum_nb", ct.c_int64),
                ("sum_nb2", ct.c_int64), ("max_nb", ct.c_int32), ("n_ops", ct.c_int32),
                ("m2m_nnz", ct.c_int64), ("lo", ct.c_double * 3), ("width", ct.c_double),
                ("mid", ct.c_double * 3), ("n_near", ct.c_int64)]


class _Flops(ct.Structure):
    _fields_ = [(k, ct.c_int64) for k in ("half", "omega", "m2m", "m2l", "l2l", "l2p", "total")]


class _JFlops(ct.Structure):
    _fields_ = [(k, ct.c_int64) for k in ("dens", "m2m", "m2l", "l2l", "pair", "total")]


class _Opts(ct.Structure):
    _fields_ = [("precision", ct.c_int32), ("rank_mode", ct.c_int32), ("selector", ct.c_void_p),
                ("jblock", ct.c_int32), ("accumulate", ct.c_int32), ("pair_thresh", ct.c_double),
                ("one_stream", ct.c_int32), ("lds_tree", ct.c_int32)]


EXPORTS = {
    "occk_abi_version": (ct.c_int32, []),
    "occk_last_error": (ct.c_char_p, []),
    "occk_build_tree": (ct.c_int32, [ct.POINTER(_System), ct.POINTER(_Params), ct.POINTER(ct.c_void_p)]),
    "occk_free_tree": (ct.c_int32, [ct.c_void_p]),
    "occk_tree_info": (ct.c_int32, [ct.c_void_p, ct.POINTER(_Info)]),
    "occk_tree_flops": (ct.c_int32, [ct.c_void_p, ct.c_int32, ct.c_int32, ct.c_int32, ct.POINTER(_Flops)]),
    "occk_tree_flops_J": (ct.c_int32, [ct.c_void_p, ct.POINTER(_JFlops)]),
    "occk_far_J": (ct.c_int32, [ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_void_p, ct.c_int64, ct.c_int32,
                                ct.c_void_p]),
    "occk_near_K": (ct.c_int32, [ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_void_p, ct.c_int64,
                                 ct.c_int32, ct.c_void_p]),
    "occk_near_info": (ct.c_int32, [ct.c_void_p, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int64)]),
    "occk_tree_near": (ct.c_int32, [ct.c_void_p, ct.c_void_p, ct.c_void_p]),
    "occk_pair_screen_info": (ct.c_int32, [ct.c_void_p, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int32),
                                           ct.c_void_p, ct.c_int32, ct.POINTER(ct.c_int32)]),
    "occk_tree_export": (ct.c_int32, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                      ct.c_void_p]),
    "occk_tree_leaf": (ct.c_int32, [ct.c_void_p, ct.c_int32, ct.POINTER(ct.c_int32), ct.c_void_p,
                                    ct.c_void_p]),
    "occk_far_K": (ct.c_int32, [ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_int32, ct.c_int32,
                                ct.c_int32, ct.c_int32, ct.POINTER(_Opts), ct.c_void_p, ct.c_int64,
                                ct.c_void_p]),
    "occk_far_K_noalloc": (ct.c_int32, [ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_int32, ct.c_int32,
                                        ct.c_int32, ct.c_int32, ct.POINTER(_Opts), ct.c_void_p, ct.c_int64,
                                        ct.c_void_p]),
    "occk_debug_mfma_probe": (ct.c_int32, [ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_void_p]),
    "occk_debug_buffer": (ct.c_int32, [ct.c_void_p, ct.c_int32, ct.c_void_p, ct.POINTER(ct.c_int64)]),
    "occk_batch_create": (ct.c_int32, [ct.c_int32, ct.c_void_p, ct.c_void_p, ct.POINTER(_Opts),
                                       ct.POINTER(ct.c_void_p)]),
    "occk_batch_run": (ct.c_int32, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p]),
    "occk_far_K_batched": (ct.c_int32, [ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                        ct.c_void_p, ct.c_void_p, ct.c_void_p]),
    "occk_batch_tune": (ct.c_int32, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                     ct.c_void_p]),
    "occk_batch_shape": (ct.c_int32, [ct.c_void_p, ct.POINTER(ct.c_int32), ct.c_void_p, ct.c_int32]),
    "occk_batch_config": (ct.c_int32, [ct.c_void_p, ct.c_void_p]),
    "occk_batch_stage_times": (ct.c_int32, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int32,
                                            ct.POINTER(ct.c_int32)]),
    "occk_batch_free": (ct.c_int32, [ct.c_void_p]),
    "occk_selector_create": (ct.c_int32, [ct.c_int32, ct.POINTER(ct.c_void_p)]),
    "occk_selector_free": (ct.c_int32, [ct.c_void_p]),
    "occk_selector_get_weights": (ct.c_int32, [ct.c_void_p, ct.c_void_p]),
    "occk_selector_set_weights": (ct.c_int32, [ct.c_void_p, ct.c_void_p]),
    "occk_selector_set_rule": (ct.c_int32, [ct.c_void_p, ct.c_float, ct.c_float]),
    "occk_selector_collect": (ct.c_int32, [ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_int32, ct.c_int32,
                                           ct.c_int32, ct.c_int32, ct.c_void_p, ct.c_void_p,
                                           ct.POINTER(ct.c_int32), ct.c_void_p]),
    "occk_selector_train": (ct.c_int32, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int32, ct.c_int32, ct.c_int32,
                                         ct.c_float, ct.c_int32, ct.c_void_p, ct.c_void_p]),
    "occk_selector_grad": (ct.c_int32, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int32, ct.POINTER(ct.c_float),
                                        ct.c_void_p, ct.c_void_p]),
    "occk_selector_predict": (ct.c_int32, [ct.c_void_p, ct.c_void_p, ct.c_int32, ct.c_int32, ct.c_void_p, ct.c_void_p,
                                           ct.c_void_p]),
    "occk_selector_save": (ct.c_int32, [ct.c_void_p, ct.c_char_p]),
    "occk_selector_load": (ct.c_int32, [ct.c_void_p, ct.c_char_p]),
    "occk_rank_stats": (ct.c_int32, [ct.c_void_p, ct.c_void_p]),
    "occk_workspace_info": (ct.c_int32, [ct.c_void_p, ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int64)]),
    "occk_profile_enable": (ct.c_int32, [ct.c_void_p, ct.c_int32]),
    "occk_profile_read": (ct.c_int32, [ct.c_void_p, ct.c_void_p, ct.c_void_p]),
}

KERNEL_CLASSES = ["opgen", "half", "omega", "up", "down", "l2p", "reduce", "convert", "select",
                  "ht", "up_walk", "down_walk", "l2p_direct", "l2p_mirror", "tree"]
NFEAT, NOUT, NPARAM = 24, 8, 6280

_lib = None


def lib():
    """Loads libocck.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is missing: build it with "
                              "`python -m paper_1708_05353_amd.build` (no CPU fallback exists)")
        L = ct.CDLL(_LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(code: int):
    if code != OK:
        raise OcckError(code, lib().occk_last_error().decode())


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ct.POINTER(ctype))


@dataclass
class TreeInfo:
    nbasis: int
    lmax: int
    ncomp: int
    depth: int
    lmin: int
    nleaf: int
    nbox: int
    boxes_per_level: list
    il_per_level: list
    n_il: int
    n_edges: int
    npairs: int
    sum_nb: int
    sum_nb2: int
    max_nb: int
    n_ops: int
    m2m_nnz: int
    lo: tuple
    width: float
    mid: tuple
    n_near: int


class Tree:
    """Handle of occk_build_tree (Step 1: pairs, boxes, lists, AO multipoles)."""

    def __init__(self, system, params):
        L = lib()
        xyz = np.ascontiguousarray(system.xyz, dtype=np.float64)
        sa = np.ascontiguousarray(system.shell_atom, dtype=np.int32)
        sl = np.ascontiguousarray(system.shell_l, dtype=np.int32)
        se = np.ascontiguousarray(system.shell_exp, dtype=np.float64)
        s = _System(int(xyz.shape[0]), _ptr(xyz, ct.c_double), int(sl.shape[0]), _ptr(sa, ct.c_int32),
                    _ptr(sl, ct.c_int32), _ptr(se, ct.c_double))
        p = _Params(int(params.split_mask), int(params.depth), int(params.ws), int(params.lmax),
                    float(params.pair_log_thresh), int(getattr(params, "near_rule", 0)),
                    float(getattr(params, "ext_ws", 0.0)), float(getattr(params, "ext_tau", 1e-8)))
        h = ct.c_void_p()
        _check(L.occk_build_tree(ct.byref(s), ct.byref(p), ct.byref(h)))
        self._h = h
        self.info = self._info()

    def _info(self) -> TreeInfo:
        inf = _Info()
        _check(lib().occk_tree_info(self._h, ct.byref(inf)))
        return TreeInfo(inf.nbasis, inf.lmax, inf.ncomp, inf.depth, inf.lmin, inf.nleaf, inf.nbox,
                        list(inf.boxes_per_level)[: inf.depth + 1], list(inf.il_per_level)[: inf.depth + 1],
                        inf.n_il, inf.n_edges, inf.npairs, inf.sum_nb, inf.sum_nb2, inf.max_nb, inf.n_ops,
                        inf.m2m_nnz, tuple(inf.lo), inf.width, tuple(inf.mid), inf.n_near)

    @property
    def handle(self):
        return self._h

    def export(self):
        inf = self.info
        leaf = np.zeros((inf.nleaf, 3), np.int32)
        lev = np.zeros(inf.n_il, np.int32)
        tgt = np.zeros(inf.n_il, np.int32)
        src = np.zeros(inf.n_il, np.int32)
        pl = np.zeros(inf.npairs, np.int32)
        _check(lib().occk_tree_export(self._h, leaf.ctypes.data, lev.ctypes.data, tgt.ctypes.data,
                                      src.ctypes.data, pl.ctypes.data))
        return leaf, lev, tgt, src, pl

    def near(self):
        """The near field: for every leaf, the sorted list of leaves near it."""
        inf = self.info
        ptr = np.zeros(inf.nleaf + 1, np.int32)
        idx = np.zeros(max(1, inf.n_near), np.int32)
        _check(lib().occk_tree_near(self._h, ptr.ctypes.data, idx.ctypes.data))
        return [idx[ptr[b]:ptr[b + 1]].tolist() for b in range(inf.nleaf)]

    def leaf(self, b: int):
        nb = ct.c_int32()
        _check(lib().occk_tree_leaf(self._h, int(b), ct.byref(nb), None, None))
        f = np.zeros(nb.value, np.int32)
        O = np.zeros((self.info.ncomp, nb.value, nb.value))
        _check(lib().occk_tree_leaf(self._h, int(b), ct.byref(nb), f.ctypes.data, O.ctypes.data))
        return f, O

    def debug_buffer(self, which: int) -> np.ndarray:
        n = ct.c_int64()
        _check(lib().occk_debug_buffer(self._h, int(which), None, ct.byref(n)))
        out = np.zeros(n.value)
        _check(lib().occk_debug_buffer(self._h, int(which), out.ctypes.data, ct.byref(n)))
        return out

    def workspace_jblock(self) -> int:
        jb = ct.c_int32()
        nb = ct.c_int64()
        _check(lib().occk_workspace_info(self._h, ct.byref(jb), ct.byref(nb)))
        return jb.value

    def workspace_bytes(self) -> int:
        jb = ct.c_int32()
        nb = ct.c_int64()
        _check(lib().occk_workspace_info(self._h, ct.byref(jb), ct.byref(nb)))
        return nb.value

    def profile(self, enable: bool = True):
        _check(lib().occk_profile_enable(self._h, int(bool(enable))))

    def profile_read(self) -> dict:
        ms = np.zeros(len(KERNEL_CLASSES))
        n = np.zeros(len(KERNEL_CLASSES), np.int64)
        _check(lib().occk_profile_read(self._h, ms.ctypes.data, n.ctypes.data))
        return {c: (float(ms[k]), int(n[k])) for k, c in enumerate(KERNEL_CLASSES)}

    def rank_stats(self) -> np.ndarray:
        h = np.zeros(9, np.int64)
        _check(lib().occk_rank_stats(self._h, h.ctypes.data))
        return h

    def free(self):
        if self._h is not None and self._h.value:
            _check(lib().occk_free_tree(self._h))
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    # ------------------------------------------------------------------
    def flops_J(self) -> dict:
        """Algorithmic flop counts of one occk_far_J call (occk_tree_flops_J)."""
        f = _JFlops()
        _check(lib().occk_tree_flops_J(self._h, ct.byref(f)))
        return {k: int(getattr(f, k)) for k, _ in _JFlops._fields_}

    def flops(self, ni: int, nj: int, symmetric: bool = False) -> dict:
        """Algorithmic flop counts of one occk_far_K call (occk_tree_flops).

        symmetric=False: paper-as-written, all ni*nj (j, i) columns carried.
        symmetric=True (i and j over the same n orbitals): n(n+1)/2 columns."""
        f = _Flops()
        _check(lib().occk_tree_flops(self._h, int(ni), int(nj), int(bool(symmetric)), ct.byref(f)))
        return {k: int(getattr(f, k)) for k, _ in _Flops._fields_}


def far_K(tree: Tree, C, K, i_range=None, j_range=None, precision: int = PREC_FP64,
          jblock: int = 0, accumulate: bool = False, stream=None, selector=None, pair_thresh: float = 0.0,
          one_stream: bool = False, lds_tree: bool = False):
    """K[:, i0:i1] (+)= 2 sum_{j in [j0,j1)} (rj|ji)_ff on the GPU.

    C: torch.float64 CUDA tensor (nbasis, ldc) row-major; K: torch.float64 CUDA
    tensor (nbasis, ldk).  Asynchronous on ``stream`` (default: torch's current
    stream).  lds_tree=True runs the translations of chain-like trees as the
    in-LDS tree kernel (occk_far_opts.lds_tree)."""
    import torch
    nocc = int(C.shape[1])
    i0, i1 = (0, nocc) if i_range is None else i_range
    j0, j1 = (0, nocc) if j_range is None else j_range
    for t in (C, K):
        if not (t.is_cuda and t.dtype == torch.float64 and t.dim() == 2 and t.stride(1) == 1):
            raise ValueError("C and K must be row-major 2-D float64 CUDA tensors")
    if stream is None:
        stream = torch.cuda.current_stream(C.device)
    opts = _Opts(int(precision), RANK_FIXED if selector is None else RANK_LEARNED,
                 None if selector is None else selector.handle.value, int(jblock), int(bool(accumulate)),
                 float(pair_thresh), int(bool(one_stream)), int(bool(lds_tree)))
    _check(lib().occk_far_K(tree.handle, ct.c_void_p(C.data_ptr()), int(C.stride(0)), nocc, int(i0), int(i1),
                            int(j0), int(j1), ct.byref(opts), ct.c_void_p(K.data_ptr()), int(K.stride(0)),
                            ct.c_void_p(stream.cuda_stream)))


def far_K_noalloc(tree: Tree, C, K, i_range=None, j_range=None, jblock: int = 0, accumulate: bool = False,
                  stream=None):
    """occk_far_K_noalloc: FP64, fixed rank, workspace in the library's fixed
    scratch region (no device allocation).  Same tensors as far_K."""
    import torch
    nocc = int(C.shape[1])
    i0, i1 = (0, nocc) if i_range is None else i_range
    j0, j1 = (0, nocc) if j_range is None else j_range
    for t in (C, K):
        if not (t.is_cuda and t.dtype == torch.float64 and t.dim() == 2 and t.stride(1) == 1):
            raise ValueError("C and K must be row-major 2-D float64 CUDA tensors")
    if stream is None:
        stream = torch.cuda.current_stream(C.device)
    opts = _Opts(PREC_FP64, RANK_FIXED, None, int(jblock), int(bool(accumulate)))
    _check(lib().occk_far_K_noalloc(tree.handle, ct.c_void_p(C.data_ptr()), int(C.stride(0)), nocc, int(i0),
                                    int(i1), int(j0), int(j1), ct.byref(opts), ct.c_void_p(K.data_ptr()),
                                    int(K.stride(0)), ct.c_void_p(stream.cuda_stream)))


def far_J(tree: Tree, D, J, accumulate: bool = False, stream=None):
    """J (+)= J^ff of the density D on the GPU (occk_far_J).  D, J: row-major
    float64 CUDA tensors (nbasis, ld); asynchronous on ``stream``."""
    import torch
    for t in (D, J):
        if not (t.is_cuda and t.dtype == torch.float64 and t.dim() == 2 and t.stride(1) == 1):
            raise ValueError("D and J must be row-major 2-D float64 CUDA tensors")
    if stream is None:
        stream = torch.cuda.current_stream(D.device)
    _check(lib().occk_far_J(tree.handle, ct.c_void_p(D.data_ptr()), int(D.stride(0)), ct.c_void_p(J.data_ptr()),
                            int(J.stride(0)), int(bool(accumulate)), ct.c_void_p(stream.cuda_stream)))


def near_K(tree: Tree, C, K, accumulate: bool = False, stream=None):
    """K (+)= K^nf of the occupied orbitals C on the GPU (occk_near_K).  C, K:
    row-major float64 CUDA tensors (nbasis, ld); asynchronous on ``stream``."""
    import torch
    for t in (C, K):
        if not (t.is_cuda and t.dtype == torch.float64 and t.dim() == 2 and t.stride(1) == 1):
            raise ValueError("C and K must be row-major 2-D float64 CUDA tensors")
    if stream is None:
        stream = torch.cuda.current_stream(C.device)
    _check(lib().occk_near_K(tree.handle, ct.c_void_p(C.data_ptr()), int(C.stride(0)), int(C.shape[1]),
                             ct.c_void_p(K.data_ptr()), int(K.stride(0)), int(bool(accumulate)),
                             ct.c_void_p(stream.cuda_stream)))


def pair_screen_info(tree: Tree) -> tuple:
    """(carried (j, i) columns, j batch width, i end of every j batch) of the
    handle's last screened occk_far_K call."""
    n, jb, nb = ct.c_int64(), ct.c_int32(), ct.c_int32()
    _check(lib().occk_pair_screen_info(tree.handle, ct.byref(n), ct.byref(jb), None, 0, ct.byref(nb)))
    ends = np.zeros(nb.value, dtype=np.int32)
    if nb.value:
        _check(lib().occk_pair_screen_info(tree.handle, ct.byref(n), ct.byref(jb), ends.ctypes.data, nb.value,
                                           ct.byref(nb)))
    return n.value, jb.value, ends


def near_info(tree: Tree) -> tuple:
    """(wave tasks, shell quartets) of one occk_near_K call on the tree."""
    a, b = ct.c_int64(), ct.c_int64()
    _check(lib().occk_near_info(tree.handle, ct.byref(a), ct.byref(b)))
    return a.value, b.value


def debug_mfma_probe(kind: int, ia: int, ka: int, jb: int) -> np.ndarray:
    out = np.zeros((64, 4))
    _check(lib().occk_debug_mfma_probe(int(kind), int(ia), int(ka), int(jb), out.ctypes.data))
    return out


class Batch:
    """Many systems in one persistent launch (occk_batch_*)."""

    def __init__(self, trees, noccs, precision: int = PREC_FP32, jblock: int = 0):
        self.trees = list(trees)
        arr = (ct.c_void_p * len(self.trees))(*[t.handle.value for t in self.trees])
        no = np.ascontiguousarray(noccs, dtype=np.int32)
        opts = _Opts(int(precision), RANK_FIXED, None, int(jblock), 0)
        h = ct.c_void_p()
        _check(lib().occk_batch_create(len(self.trees), ct.cast(arr, ct.c_void_p), no.ctypes.data, ct.byref(opts),
                                       ct.byref(h)))
        self._h = h
        self.noccs = [int(x) for x in no]

    def _io(self, Cs, Ks):
        n = len(self.trees)
        self._keep = (
            (ct.c_void_p * n)(*[c.data_ptr() for c in Cs]),
            np.array([c.stride(0) for c in Cs], np.int64),
            (ct.c_void_p * n)(*[k.data_ptr() for k in Ks]),
            np.array([k.stride(0) for k in Ks], np.int64),
        )
        a, b, c, d = self._keep
        return ct.cast(a, ct.c_void_p), b.ctypes.data, ct.cast(c, ct.c_void_p), d.ctypes.data

    def stage_times(self):
        """(ms per stage, task type per stage) of the last launch."""
        n = ct.c_int32()
        _check(lib().occk_batch_stage_times(self._h, None, None, 0, ct.byref(n)))
        ms = np.zeros(max(1, n.value), np.float64)
        ty = np.zeros(max(1, n.value), np.int32)
        _check(lib().occk_batch_stage_times(self._h, ms.ctypes.data, ty.ctypes.data, n.value, ct.byref(n)))
        return ms[:n.value], ty[:n.value]

    def run(self, Cs, Ks, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        _check(lib().occk_batch_run(self._h, *self._io(Cs, Ks), ct.c_void_p(stream.cuda_stream)))

    def tune(self, Cs, Ks, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        ch = np.zeros(3, np.int32)
        _check(lib().occk_batch_tune(self._h, *self._io(Cs, Ks), ct.c_void_p(stream.cuda_stream), ch.ctypes.data))
        return tuple(int(x) for x in ch)

    def config(self):
        c = np.zeros(6, np.int32)
        _check(lib().occk_batch_config(self._h, c.ctypes.data))
        return dict(blocks_per_cu=int(c[0]), gemm_group=int(c[1]), trans_group=int(c[2]), ntasks=int(c[3]),
                    nstage=int(c[4]), max_blocks_per_cu=int(c[5]))

    def free(self):
        if self._h is not None and self._h.value:
            _check(lib().occk_batch_free(self._h))
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def far_K_batched(trees, Cs, Ks, precision: int = PREC_FP32, jblock: int = 0, stream=None):
    """K^ff of every system in one persistent launch (occk_far_K_batched: a
    plan made, run and freed in one call; returns after the launch)."""
    import torch
    n = len(trees)
    if not (len(Cs) == len(Ks) == n):
        raise ValueError("one C and one K per tree")
    if stream is None:
        stream = torch.cuda.current_stream()
    th = (ct.c_void_p * n)(*[t.handle.value for t in trees])
    cp = (ct.c_void_p * n)(*[c.data_ptr() for c in Cs])
    kp = (ct.c_void_p * n)(*[k.data_ptr() for k in Ks])
    ldc = np.array([c.stride(0) for c in Cs], np.int64)
    ldk = np.array([k.stride(0) for k in Ks], np.int64)
    no = np.array([c.shape[1] for c in Cs], np.int32)
    opts = _Opts(int(precision), RANK_FIXED, None, int(jblock), 0)
    _check(lib().occk_far_K_batched(n, ct.cast(th, ct.c_void_p), ct.cast(cp, ct.c_void_p), ldc.ctypes.data,
                                    no.ctypes.data, ct.byref(opts), ct.cast(kp, ct.c_void_p), ldk.ctypes.data,
                                    ct.c_void_p(stream.cuda_stream)))


class Selector:
    """Learned rank per interaction-list translation (occk_selector_*)."""

    def __init__(self, seed: int = 0):
        h = ct.c_void_p()
        _check(lib().occk_selector_create(int(seed), ct.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def weights(self) -> np.ndarray:
        w = np.zeros(NPARAM, np.float32)
        _check(lib().occk_selector_get_weights(self._h, w.ctypes.data))
        return w

    def set_weights(self, w):
        w = np.ascontiguousarray(w, np.float32)
        _check(lib().occk_selector_set_weights(self._h, w.ctypes.data))

    def set_rule(self, log10_tau: float, margin: float):
        _check(lib().occk_selector_set_rule(self._h, float(log10_tau), float(margin)))

    @staticmethod
    def collect(tree: Tree, C, j_range, max_samples: int, seed: int = 0, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(C.device)
        X = np.zeros((max_samples, NFEAT), np.float32)
        T = np.zeros((max_samples, NOUT), np.float32)
        n = ct.c_int32()
        _check(lib().occk_selector_collect(tree.handle, ct.c_void_p(C.data_ptr()), int(C.stride(0)), int(C.shape[1]),
                                           int(j_range[0]), int(j_range[1]), int(max_samples), int(seed),
                                           X.ctypes.data, T.ctypes.data, ct.byref(n), ct.c_void_p(stream.cuda_stream)))
        return X[: n.value].copy(), T[: n.value].copy()

    def train(self, X, T, epochs=20, batch=512, lr=1e-3, seed=0, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        X = np.ascontiguousarray(X, np.float32)
        T = np.ascontiguousarray(T, np.float32)
        loss = np.zeros(epochs, np.float32)
        _check(lib().occk_selector_train(self._h, X.ctypes.data, T.ctypes.data, int(X.shape[0]), int(epochs), int(batch),
                                         float(lr), int(seed), loss.ctypes.data, ct.c_void_p(stream.cuda_stream)))
        return loss

    def grad(self, X, T, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        X = np.ascontiguousarray(X, np.float32)
        T = np.ascontiguousarray(T, np.float32)
        g = np.zeros(NPARAM, np.float32)
        l = ct.c_float()
        _check(lib().occk_selector_grad(self._h, X.ctypes.data, T.ctypes.data, int(X.shape[0]), ct.byref(l),
                                        g.ctypes.data, ct.c_void_p(stream.cuda_stream)))
        return float(l.value), g

    def predict(self, X, lmax: int = 8, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        X = np.ascontiguousarray(X, np.float32)
        z = np.zeros((X.shape[0], NOUT), np.float32)
        r = np.zeros(X.shape[0], np.int32)
        _check(lib().occk_selector_predict(self._h, X.ctypes.data, int(X.shape[0]), int(lmax), z.ctypes.data,
                                           r.ctypes.data, ct.c_void_p(stream.cuda_stream)))
        return z, r

    def save(self, path: str):
        _check(lib().occk_selector_save(self._h, path.encode()))

    def load(self, path: str):
        _check(lib().occk_selector_load(self._h, path.encode()))

    def free(self):
        if self._h is not None and self._h.value:
            _check(lib().occk_selector_free(self._h))
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

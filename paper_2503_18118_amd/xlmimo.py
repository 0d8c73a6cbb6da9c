"""ctypes binding of libxlmimo (include/xlmimo.h): argument marshalling only.

Device buffers are torch CUDA tensors; every computation runs in the HIP
library.  Importing this module loads ``libxlmimo.so`` from the package
directory and raises if it has not been built (there is no fallback).
"""
from __future__ import annotations

import ctypes as C
import os
import weakref
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libxlmimo.so")

OK, EINVAL, EDEVICE, ENOMEM, ENOTIMPL = 0, -1, -2, -3, -4
ULA, UPA = 0, 1
AMP_FREESPACE, AMP_PNUSW = 0, 1
FP64, FP32C, FP32H = 0, 1, 2
CF_PAPER, CF_GATED, CF_UNIFORM, CF_GATED_QUAD = 0, 1, 2, 3
ZF, MMSE, MRC, CAP, MZF, MZF_MISM, CORR_GAP = 1, 2, 4, 8, 16, 32, 64
ST_G_NOT_PD, ST_MMSE_NOT_PD, ST_FILTER_NOT_PD, ST_BAD_INPUT, ST_CF_DEGENERATE, ST_FELL_BACK = 1, 2, 4, 8, 16, 32
FORM_EXACT_FP64, FORM_EXACT_FP32C, FORM_CF_PAPER, FORM_CF_GATED, FORM_CF_GATED_MLP, FORM_EXACT_FP32H, FORM_CF_UNIFORM = \
    0, 1, 2, 3, 4, 5, 6
MAX_USERS, MAX_USERS_EXACT = 64, 1024
MLP_IN, MLP_OUT, PAIR_FEAT_PITCH, PAIR_AUX_PITCH = 6, 7, 8, 8

EXPORTED = ("xlmimo_ctx_create", "xlmimo_ctx_destroy", "xlmimo_last_error", "xlmimo_version",
            "xlmimo_gram_exact", "xlmimo_gram_closedform", "xlmimo_zf_mmse_sumrate",
            "xlmimo_capacity_sweep", "xlmimo_timing_enable", "xlmimo_timing_read",
            "xlmimo_mlp_create", "xlmimo_mlp_destroy", "xlmimo_mlp_param_count", "xlmimo_mlp_set_params",
            "xlmimo_mlp_get_params", "xlmimo_pair_count", "xlmimo_mlp_pair_inputs", "xlmimo_mlp_loss_grad",
            "xlmimo_mlp_train_step", "xlmimo_mlp_forward", "xlmimo_gram_closedform_mlp",
            "xlmimo_graph_begin", "xlmimo_graph_end", "xlmimo_graph_launch", "xlmimo_graph_node_count",
            "xlmimo_graph_destroy", "xlmimo_autotune_exact", "xlmimo_gram_update_users", "xlmimo_cholesky",
            "xlmimo_cholesky_update_users", "xlmimo_gram_exact_noalloc", "xlmimo_mlp_set_gate",
            "xlmimo_mlp_train")


class XlArray(C.Structure):
    _fields_ = [("geometry", C.c_int32), ("amp_model", C.c_int32), ("n_y", C.c_int64), ("n_z", C.c_int64),
                ("spacing_m", C.c_double), ("wavelength_m", C.c_double), ("beta0", C.c_double)]


class XlBatch(C.Structure):
    _fields_ = [("n_drops", C.c_int64), ("n_elems", C.POINTER(C.c_int64)), ("n_users", C.POINTER(C.c_int32)),
                ("user_pos", C.c_void_p)]


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build() "
                          "(the HIP library is required; there is no CPU fallback)")
    lib = C.CDLL(path)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    lib.xlmimo_ctx_create.argtypes = [C.POINTER(vp), C.c_int]
    lib.xlmimo_ctx_destroy.argtypes = [vp]
    lib.xlmimo_last_error.argtypes = [vp]
    lib.xlmimo_last_error.restype = C.c_char_p
    lib.xlmimo_version.restype = C.c_char_p
    lib.xlmimo_gram_exact.argtypes = [vp, C.POINTER(XlArray), C.POINTER(XlBatch), i32, vp, vp]
    lib.xlmimo_gram_exact_noalloc.argtypes = [vp, C.POINTER(XlArray), C.POINTER(XlBatch), i32, vp, vp]
    lib.xlmimo_gram_update_users.argtypes = [vp, C.POINTER(XlArray), C.POINTER(XlBatch), i32, i64,
                                             C.POINTER(C.c_int64), vp, vp]
    lib.xlmimo_cholesky.argtypes = [vp, C.POINTER(XlBatch), vp, vp, vp, vp, vp, vp]
    lib.xlmimo_cholesky_update_users.argtypes = [vp, C.POINTER(XlArray), C.POINTER(XlBatch), i64,
                                                 C.POINTER(C.c_int64), vp, vp, vp, vp, vp, vp]
    lib.xlmimo_gram_closedform.argtypes = [vp, C.POINTER(XlArray), C.POINTER(XlBatch), i32, vp, vp, vp]
    lib.xlmimo_zf_mmse_sumrate.argtypes = [vp, C.POINTER(XlBatch), vp, vp, i32, vp, i32, vp, vp, vp]
    lib.xlmimo_capacity_sweep.argtypes = [vp, C.POINTER(XlArray), i32, C.POINTER(C.c_int64), C.POINTER(XlBatch),
                                          i32, vp, C.c_double, i32, vp, i32, C.c_double, C.c_double, vp, vp, vp, vp]
    lib.xlmimo_mlp_create.argtypes = [vp, i32, i32, C.POINTER(vp)]
    lib.xlmimo_mlp_destroy.argtypes = [vp]
    lib.xlmimo_mlp_param_count.argtypes = [vp]
    lib.xlmimo_mlp_param_count.restype = i64
    lib.xlmimo_mlp_set_params.argtypes = [vp, vp]
    lib.xlmimo_mlp_get_params.argtypes = [vp, vp]
    lib.xlmimo_mlp_set_gate.argtypes = [vp, i32, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
    lib.xlmimo_pair_count.argtypes = [C.POINTER(XlBatch)]
    lib.xlmimo_pair_count.restype = i64
    lib.xlmimo_mlp_pair_inputs.argtypes = [vp, C.POINTER(XlArray), C.POINTER(XlBatch), vp, vp, vp, vp, vp, vp, vp]
    lib.xlmimo_mlp_loss_grad.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp]
    lib.xlmimo_mlp_train_step.argtypes = [vp, vp, i64, vp, vp, vp, C.c_float, vp, vp]
    lib.xlmimo_mlp_forward.argtypes = [vp, vp, i64, vp, vp, vp]
    lib.xlmimo_mlp_train.argtypes = [vp, vp, i64, vp, vp, vp, i64, i64, vp, vp, vp]
    lib.xlmimo_gram_closedform_mlp.argtypes = [vp, C.POINTER(XlArray), C.POINTER(XlBatch), i32, vp, C.c_double, vp,
                                               vp, vp]
    lib.xlmimo_timing_enable.argtypes = [vp, C.c_int]
    lib.xlmimo_timing_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    lib.xlmimo_graph_begin.argtypes = [vp, vp]
    lib.xlmimo_graph_end.argtypes = [vp, vp, C.POINTER(vp)]
    lib.xlmimo_graph_launch.argtypes = [vp, vp]
    lib.xlmimo_graph_node_count.argtypes = [vp]
    lib.xlmimo_graph_node_count.restype = i64
    lib.xlmimo_graph_destroy.argtypes = [vp]
    lib.xlmimo_autotune_exact.argtypes = [vp, C.POINTER(XlArray), C.POINTER(XlBatch), i64, i32,
                                          C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_double), vp]
    return lib


_lib = load_library()


class XlmimoError(RuntimeError):
    pass


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device buffers must be CUDA tensors")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def make_array(arr) -> XlArray:
    """workloads.ArraySpec -> struct xlmimo_array."""
    return XlArray(int(arr.geometry), int(arr.amp_model), int(arr.n_y), int(arr.n_z),
                   float(arr.spacing), float(arr.wavelength), float(arr.beta0))


class Batch:
    """Host descriptors + device positions of a workloads.Drops batch (kept alive together)."""

    def __init__(self, drops, pos: Optional[torch.Tensor] = None, device: int = 0, use_n_elems: bool = True):
        self.n_drops = drops.n_drops
        self.n_elems = np.ascontiguousarray(drops.n_elems, np.int64)
        self.n_users = np.ascontiguousarray(drops.n_users, np.int32)
        self.total_users = int(drops.user_off[-1])
        self.k = self.n_users.astype(np.int64)
        self.gram_off = np.concatenate([[0], np.cumsum(self.k * self.k)]).astype(np.int64)
        self.user_off = np.asarray(drops.user_off, np.int64)
        if pos is None:
            pos = torch.as_tensor(np.ascontiguousarray(drops.pos, np.float64), device=f"cuda:{device}")
        self.pos = pos.contiguous()
        self.struct = XlBatch(self.n_drops,
                              self.n_elems.ctypes.data_as(C.POINTER(C.c_int64)) if use_n_elems else None,
                              self.n_users.ctypes.data_as(C.POINTER(C.c_int32)),
                              C.c_void_p(self.pos.data_ptr()) if self.total_users else None)

    @property
    def gram_elems(self) -> int:
        return int(self.gram_off[-1])

    def split(self, flat: torch.Tensor) -> list:
        """Split a flat complex128 Gram buffer into per-drop K x K numpy arrays."""
        g = flat.detach().cpu().numpy().view(np.complex128)
        return [g[self.gram_off[d]:self.gram_off[d + 1]].reshape(self.k[d], self.k[d]) for d in range(self.n_drops)]


class Context:
    def __init__(self, device: int = 0):
        self.device = device
        h = C.c_void_p()
        rc = _lib.xlmimo_ctx_create(C.byref(h), device)
        if rc != OK:
            raise XlmimoError(f"xlmimo_ctx_create failed ({rc})")
        self.h = h
        self._children = weakref.WeakSet()   # MLPs of this context, destroyed before it

    def close(self):
        if getattr(self, "h", None):
            # graphs first, then networks, then the context
            for child in sorted(self._children, key=lambda c: not isinstance(c, Graph)):
                child.close()
            _lib.xlmimo_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int, what: str):
        if rc != OK:
            msg = _lib.xlmimo_last_error(self.h)
            raise XlmimoError(f"{what} failed ({rc}): {msg.decode() if msg else ''}")

    # -- benchmark timing of the exact-Gram kernel ----------------------------
    def timing_enable(self, on: bool = True):
        self._check(_lib.xlmimo_timing_enable(self.h, 1 if on else 0), "xlmimo_timing_enable")

    def timing_read(self):
        ms, n = C.c_double(), C.c_int64()
        self._check(_lib.xlmimo_timing_read(self.h, C.byref(ms), C.byref(n)), "xlmimo_timing_read")
        return ms.value, n.value

    # -- batching: graph capture and autotuning ---------------------------------
    def graph_begin(self, stream):
        """Open a capture on `stream` (a torch.cuda.Stream other than the default one)."""
        self._check(_lib.xlmimo_graph_begin(self.h, _stream(stream)), "xlmimo_graph_begin")

    def graph_end(self, stream) -> "Graph":
        h = C.c_void_p()
        self._check(_lib.xlmimo_graph_end(self.h, _stream(stream), C.byref(h)), "xlmimo_graph_end")
        return Graph(self, h)

    def autotune_exact(self, arr, batch: "Batch", precision: int = FP32H, n_elems: int = 0, stream=None) -> dict:
        ch, g, ms = C.c_int64(), C.c_int32(), C.c_double()
        a = make_array(arr)
        self._check(_lib.xlmimo_autotune_exact(self.h, C.byref(a), C.byref(batch.struct), int(n_elems), precision,
                                               C.byref(ch), C.byref(g), C.byref(ms), _stream(stream)),
                    "xlmimo_autotune_exact")
        return {"chunk": ch.value, "grid": g.value, "ms": ms.value}

    # -- entry points ------------------------------------------------------
    def gram_exact(self, arr, batch: Batch, precision: int = FP32C, out: Optional[torch.Tensor] = None,
                   stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(2 * batch.gram_elems, dtype=torch.float64, device=batch.pos.device)
        a = make_array(arr)
        self._check(_lib.xlmimo_gram_exact(self.h, C.byref(a), C.byref(batch.struct), precision, _ptr(out),
                                           _stream(stream)), "xlmimo_gram_exact")
        return out

    def gram_exact_noalloc(self, arr, batch: Batch, precision: int, out: torch.Tensor, stream=None) -> torch.Tensor:
        """xlmimo_gram_exact_noalloc into the caller's `out` (complex128 interleaved, the Gram layout)."""
        a = make_array(arr)
        self._check(_lib.xlmimo_gram_exact_noalloc(self.h, C.byref(a), C.byref(batch.struct), precision, _ptr(out),
                                                   _stream(stream)), "xlmimo_gram_exact_noalloc")
        return out

    def gram_update_users(self, arr, batch: Batch, moved, gram: torch.Tensor, precision: int = FP32C,
                          stream=None) -> torch.Tensor:
        """Recompute, in place, the rows and columns of `gram` that involve the users `moved`
        (global indices, strictly ascending) after their positions in batch.pos changed."""
        mv = np.ascontiguousarray(moved, np.int64)
        a = make_array(arr)
        self._check(_lib.xlmimo_gram_update_users(self.h, C.byref(a), C.byref(batch.struct), precision, len(mv),
                                                  mv.ctypes.data_as(C.POINTER(C.c_int64)), _ptr(gram),
                                                  _stream(stream)), "xlmimo_gram_update_users")
        return gram

    def cholesky(self, batch: Batch, gram: torch.Tensor, rho: Optional[torch.Tensor] = None, stream=None):
        """Factors L of G (or of I + D^1/2 G D^1/2 for one SNR row rho), LAPACK column-major per drop.
        Returns (factor, log2 det, status)."""
        factor = torch.empty_like(gram)
        logdet = torch.empty(batch.n_drops, dtype=torch.float64, device=gram.device)
        status = torch.empty(batch.n_drops, dtype=torch.int32, device=gram.device)
        r = None if rho is None else rho.contiguous()
        self._check(_lib.xlmimo_cholesky(self.h, C.byref(batch.struct), _ptr(gram), _ptr(r), _ptr(factor),
                                         _ptr(logdet), _ptr(status), _stream(stream)), "xlmimo_cholesky")
        return factor, logdet, status

    def cholesky_update_users(self, arr, batch: Batch, moved, gram: torch.Tensor, factor: torch.Tensor,
                              rho: Optional[torch.Tensor] = None, logdet: Optional[torch.Tensor] = None,
                              status: Optional[torch.Tensor] = None, stream=None):
        """Update `factor` in place after the rows of `moved` changed in `gram`; returns (logdet, status)."""
        mv = np.ascontiguousarray(moved, np.int64)
        if logdet is None:
            logdet = torch.full((batch.n_drops,), float("nan"), dtype=torch.float64, device=gram.device)
        if status is None:
            status = torch.zeros(batch.n_drops, dtype=torch.int32, device=gram.device)
        a = make_array(arr)
        r = None if rho is None else rho.contiguous()
        self._check(_lib.xlmimo_cholesky_update_users(self.h, C.byref(a), C.byref(batch.struct), len(mv),
                                                      mv.ctypes.data_as(C.POINTER(C.c_int64)), _ptr(gram), _ptr(r),
                                                      _ptr(factor), _ptr(logdet), _ptr(status), _stream(stream)),
                    "xlmimo_cholesky_update_users")
        return logdet, status

    def gram_closedform(self, arr, batch: Batch, variant: int = CF_PAPER, out: Optional[torch.Tensor] = None,
                        status: Optional[torch.Tensor] = None, stream=None):
        if out is None:
            out = torch.empty(2 * batch.gram_elems, dtype=torch.float64, device=batch.pos.device)
        if status is None:
            status = torch.empty(batch.n_drops, dtype=torch.int32, device=batch.pos.device)
        a = make_array(arr)
        self._check(_lib.xlmimo_gram_closedform(self.h, C.byref(a), C.byref(batch.struct), variant, _ptr(out),
                                                _ptr(status), _stream(stream)), "xlmimo_gram_closedform")
        return out, status

    def sumrate(self, batch: Batch, gram_true: torch.Tensor, rho: torch.Tensor, schemes: int = ZF | MMSE,
                gram_filter: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
                status: Optional[torch.Tensor] = None, stream=None):
        """rho: CUDA float64 [n_snr, total_users].  Returns (rates [n_drops, n_snr, n_sch], status)."""
        n_snr = int(rho.shape[0])
        n_sch = bin(schemes).count("1")
        if out is None:
            out = torch.empty((batch.n_drops, n_snr, n_sch), dtype=torch.float64, device=gram_true.device)
        if status is None:
            status = torch.empty(batch.n_drops, dtype=torch.int32, device=gram_true.device)
        self._check(_lib.xlmimo_zf_mmse_sumrate(self.h, C.byref(batch.struct), _ptr(gram_true), _ptr(gram_filter),
                                                n_snr, _ptr(rho.contiguous()), schemes, _ptr(out), _ptr(status),
                                                _stream(stream)), "xlmimo_zf_mmse_sumrate")
        return out, status

    def capacity_sweep(self, arr, n_list: Sequence[int], batch: Batch, form: int, rho: torch.Tensor,
                       schemes: int = ZF | MMSE, t_sat: float = 0.9, eps_sat: float = 0.05,
                       ergodic: Optional[torch.Tensor] = None, sat: Optional[torch.Tensor] = None,
                       status: Optional[torch.Tensor] = None, stream=None, mlp=None, log_var_max: float = 0.0):
        n_snr = int(rho.shape[0])
        n_sch = bin(schemes).count("1")
        dev = batch.pos.device
        nl = np.ascontiguousarray(n_list, np.int64)
        if ergodic is None:
            ergodic = torch.empty((len(nl), n_snr, n_sch), dtype=torch.float64, device=dev)
        if sat is None:
            sat = torch.empty(3 + n_snr * n_sch, dtype=torch.float64, device=dev)
        if status is None:
            status = torch.empty((len(nl), batch.n_drops), dtype=torch.int32, device=dev)
        a = make_array(arr)
        self._check(_lib.xlmimo_capacity_sweep(self.h, C.byref(a), len(nl), nl.ctypes.data_as(C.POINTER(C.c_int64)),
                                               C.byref(batch.struct), form, mlp.h if mlp is not None else None,
                                               float(log_var_max), n_snr, _ptr(rho.contiguous()), schemes,
                                               float(t_sat), float(eps_sat), _ptr(ergodic), _ptr(sat), _ptr(status),
                                               _stream(stream)), "xlmimo_capacity_sweep")
        return ergodic, sat, status


    def gram_closedform_mlp(self, arr, batch: "Batch", mlp, variant: int = CF_GATED, log_var_max: float = 0.0,
                            out: Optional[torch.Tensor] = None, status: Optional[torch.Tensor] = None, stream=None):
        if out is None:
            out = torch.empty(2 * batch.gram_elems, dtype=torch.float64, device=batch.pos.device)
        if status is None:
            status = torch.empty(batch.n_drops, dtype=torch.int32, device=batch.pos.device)
        a = make_array(arr)
        self._check(_lib.xlmimo_gram_closedform_mlp(self.h, C.byref(a), C.byref(batch.struct), variant, mlp.h,
                                                    float(log_var_max), _ptr(out), _ptr(status), _stream(stream)),
                    "xlmimo_gram_closedform_mlp")
        return out, status


class Graph:
    """Executable graph of library calls captured with Context.graph_begin / graph_end."""

    def __init__(self, ctx: Context, h):
        self.ctx, self.h = ctx, h
        ctx._children.add(self)

    @property
    def n_nodes(self) -> int:
        return int(_lib.xlmimo_graph_node_count(self.h))

    def launch(self, stream=None):
        self.ctx._check(_lib.xlmimo_graph_launch(self.h, _stream(stream)), "xlmimo_graph_launch")

    def close(self):
        if getattr(self, "h", None) and getattr(self.ctx, "h", None):
            _lib.xlmimo_graph_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PairInputs:
    """Per-pair network inputs (device): bf16 features, float aux, optional targets, pair map."""

    def __init__(self, feat, aux, target, pmap):
        self.feat, self.aux, self.target, self.pmap = feat, aux, target, pmap

    @property
    def n(self) -> int:
        return int(self.feat.shape[0])

    def slice(self, a: int, b: int) -> "PairInputs":
        return PairInputs(self.feat[a:b], self.aux[a:b], None if self.target is None else self.target[a:b],
                          self.pmap[a:b])


class MLP:
    """Device-resident network of the learned correction (include/xlmimo.h)."""

    def __init__(self, ctx: Context, width: int = 256, depth: int = 4):
        self.ctx, self.width, self.depth = ctx, width, depth
        h = C.c_void_p()
        ctx._check(_lib.xlmimo_mlp_create(ctx.h, width, depth, C.byref(h)), "xlmimo_mlp_create")
        self.h = h
        self.n_params = int(_lib.xlmimo_mlp_param_count(h))
        ctx._children.add(self)

    def close(self):
        # the context destroys its MLPs first; after that this handle is gone
        if getattr(self, "h", None) and getattr(self.ctx, "h", None):
            _lib.xlmimo_mlp_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params: np.ndarray):
        p = np.ascontiguousarray(params, np.float32)
        assert p.size == self.n_params
        self.ctx._check(_lib.xlmimo_mlp_set_params(self.h, p.ctypes.data_as(C.c_void_p)), "xlmimo_mlp_set_params")

    def get_params(self) -> np.ndarray:
        p = np.empty(self.n_params, np.float32)
        self.ctx._check(_lib.xlmimo_mlp_get_params(self.h, p.ctypes.data_as(C.c_void_p)), "xlmimo_mlp_get_params")
        return p

    def set_gate(self, n_upper: Sequence[int], log_var_max: Sequence[float]):
        """Fallback thresholds by antenna count (xlmimo_mlp_set_gate); empty lists clear the table."""
        nu = np.ascontiguousarray(n_upper, np.int64)
        th = np.ascontiguousarray(log_var_max, np.float64)
        assert nu.size == th.size
        self.ctx._check(_lib.xlmimo_mlp_set_gate(self.h, int(nu.size), nu.ctypes.data_as(C.POINTER(C.c_int64)),
                                                 th.ctypes.data_as(C.POINTER(C.c_double))), "xlmimo_mlp_set_gate")

    def pair_inputs(self, arr, batch: Batch, gram_cf: torch.Tensor, gram_exact: Optional[torch.Tensor] = None,
                    stream=None) -> PairInputs:
        n = int(_lib.xlmimo_pair_count(C.byref(batch.struct)))
        dev = gram_cf.device
        feat = torch.empty((n, PAIR_FEAT_PITCH), dtype=torch.bfloat16, device=dev)
        aux = torch.empty((n, PAIR_AUX_PITCH), dtype=torch.float32, device=dev)
        target = torch.empty((n, 2), dtype=torch.float32, device=dev) if gram_exact is not None else None
        pmap = torch.empty((n, 2), dtype=torch.int32, device=dev)
        a = make_array(arr)
        self.ctx._check(_lib.xlmimo_mlp_pair_inputs(self.ctx.h, C.byref(a), C.byref(batch.struct), _ptr(gram_cf),
                                                    _ptr(gram_exact), _ptr(feat), _ptr(aux), _ptr(target), _ptr(pmap),
                                                    _stream(stream)), "xlmimo_mlp_pair_inputs")
        return PairInputs(feat, aux, target, pmap)

    def loss_grad(self, pi: PairInputs, stream=None):
        grad = torch.empty(self.n_params, dtype=torch.float32, device=pi.aux.device)
        loss = torch.empty(1, dtype=torch.float64, device=pi.aux.device)
        self.ctx._check(_lib.xlmimo_mlp_loss_grad(self.ctx.h, self.h, pi.n, _ptr(pi.feat), _ptr(pi.aux),
                                                  _ptr(pi.target), _ptr(grad), _ptr(loss), _stream(stream)),
                        "xlmimo_mlp_loss_grad")
        return loss, grad

    def train_step(self, pi: PairInputs, lr: float, loss: Optional[torch.Tensor] = None, stream=None):
        if loss is None:
            loss = torch.empty(1, dtype=torch.float64, device=pi.aux.device)
        self.ctx._check(_lib.xlmimo_mlp_train_step(self.ctx.h, self.h, pi.n, _ptr(pi.feat), _ptr(pi.aux),
                                                   _ptr(pi.target), float(lr), _ptr(loss), _stream(stream)),
                        "xlmimo_mlp_train_step")
        return loss

    def train(self, pi: PairInputs, batch: int, lr: np.ndarray, loss: Optional[torch.Tensor] = None, stream=None):
        """len(lr) Adam steps over consecutive batch slices of pi (xlmimo_mlp_train); loss: CUDA float64
        [len(lr)] or None."""
        lr = np.ascontiguousarray(lr, np.float32)
        self.ctx._check(_lib.xlmimo_mlp_train(self.ctx.h, self.h, pi.n, _ptr(pi.feat), _ptr(pi.aux), _ptr(pi.target),
                                              int(batch), int(lr.size), lr.ctypes.data_as(C.c_void_p), _ptr(loss),
                                              _stream(stream)), "xlmimo_mlp_train")
        return loss

    def forward(self, pi: PairInputs, stream=None) -> torch.Tensor:
        out = torch.empty((pi.n, MLP_OUT), dtype=torch.float32, device=pi.aux.device)
        self.ctx._check(_lib.xlmimo_mlp_forward(self.ctx.h, self.h, pi.n, _ptr(pi.feat), _ptr(out), _stream(stream)),
                        "xlmimo_mlp_forward")
        return out


def version() -> str:
    return _lib.xlmimo_version().decode()

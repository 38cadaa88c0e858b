"""ctypes binding of libpdg (include/pdg.h), with the same function names.

The ``pdg_*`` functions only marshal arguments: device pointers are plain ints
(e.g. ``tensor.data_ptr()``), streams are ``hipStream_t`` handles as ints.  Every
step of the sampler runs in the library's HIP kernels; a missing library is an
error, never a fallback.

``Sampler`` is a convenience wrapper that keeps the inputs in torch device
tensors (torch supplies device memory and the stream, nothing else).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpdg.so")

PDG_OK, PDG_EINVAL, PDG_ENOMEM, PDG_EHIP = 0, -1, -2, -3
PDG_ENOTFOUND, PDG_ECAPACITY, PDG_ENONPOS, PDG_ESTATE = -4, -5, -6, -7
PDG_PRECISION_F32, PDG_PRECISION_F64 = 0, 1

EXPORTS = [
    "pdg_create", "pdg_destroy", "pdg_set_nodes", "pdg_insert_edges", "pdg_remove_edges",
    "pdg_num_edges", "pdg_live_uids", "pdg_decompose", "pdg_params_layout", "pdg_init_chains",
    "pdg_set_state", "pdg_get_state", "pdg_get_sweep", "pdg_set_sweep", "pdg_sweep",
    "pdg_dual_phase", "pdg_primal_phase", "pdg_get_duals", "pdg_get_marginals",
    "pdg_get_counts", "pdg_reset_marginals", "pdg_sync", "pdg_last_error", "pdg_log_v",
    "pdg_log_v_noalloc", "pdg_graph_create", "pdg_graph_launch", "pdg_graph_destroy",
    "pdg_tune", "pdg_set_tuning", "pdg_get_tuning",
]


class PdgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pdg error {code}: {msg}")
        self.code = code


class pdg_config(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("n_chains", ctypes.c_int32),
                ("q_max", ctypes.c_int32), ("node_capacity", ctypes.c_int64),
                ("edge_capacity", ctypes.c_int64), ("precision", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("burn_in", ctypes.c_int64)]


_lib = None
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32


class pdg_tuning(ctypes.Structure):
    _fields_ = [("dual_edges_per_wave", _I32), ("binary_groups_per_wave", _I32),
                ("hub_threshold", _I32), ("hub_piece", _I32),
                ("dual_ms", ctypes.c_float), ("primal_ms", ctypes.c_float)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def lib():
    """Load libpdg.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1611_06684_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        S = _I32
        sig = {
            "pdg_create": ([ctypes.POINTER(pdg_config), _I32, _P, ctypes.POINTER(_P)], S),
            "pdg_destroy": ([_P], S),
            "pdg_set_nodes": ([_P, _I64, _P, _P], S),
            "pdg_insert_edges": ([_P, _I64, _P, _P, _P, _P], S),
            "pdg_remove_edges": ([_P, _I64, _P], S),
            "pdg_num_edges": ([_P, ctypes.POINTER(_I64)], S),
            "pdg_live_uids": ([_P, _P], S),
            "pdg_decompose": ([_I64, _I32, _P, _P, _P, _I32, _P, _P], S),
            "pdg_params_layout": ([_I32] + [ctypes.POINTER(_I64)] * 5, S),
            "pdg_init_chains": ([_P], S),
            "pdg_set_state": ([_P, _P], S),
            "pdg_get_state": ([_P, _P], S),
            "pdg_get_sweep": ([_P, ctypes.POINTER(_I64)], S),
            "pdg_set_sweep": ([_P, _I64], S),
            "pdg_sweep": ([_P, _I64], S),
            "pdg_dual_phase": ([_P], S),
            "pdg_primal_phase": ([_P], S),
            "pdg_get_duals": ([_P, _I64, _P, _P], S),
            "pdg_log_v": ([_P, _P], S),
            "pdg_log_v_noalloc": ([_P, _P], S),
            "pdg_graph_create": ([ctypes.POINTER(_P), _I32, _I32, ctypes.POINTER(_P)], S),
            "pdg_graph_launch": ([_P], S),
            "pdg_graph_destroy": ([_P], S),
            "pdg_tune": ([_P, _I32, ctypes.POINTER(pdg_tuning)], S),
            "pdg_set_tuning": ([_P, ctypes.POINTER(pdg_tuning)], S),
            "pdg_get_tuning": ([_P, ctypes.POINTER(pdg_tuning)], S),
            "pdg_get_marginals": ([_P, _P, ctypes.POINTER(_I64)], S),
            "pdg_get_counts": ([_P, _P, ctypes.POINTER(_I64)], S),
            "pdg_reset_marginals": ([_P], S),
            "pdg_sync": ([_P], S),
            "pdg_last_error": ([_P], ctypes.c_char_p),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _chk(code, ctx=None):
    if code != PDG_OK:
        raise PdgError(code, pdg_last_error(ctx))


# ------------------------------------------------------------- C ABI, 1:1
def pdg_last_error(ctx=None) -> str:
    return (lib().pdg_last_error(ctx) or b"").decode()


def pdg_create(cfg: pdg_config, device: int = 0, stream: int = 0):
    out = _P()
    _chk(lib().pdg_create(ctypes.byref(cfg), device, stream, ctypes.byref(out)))
    return out


def pdg_destroy(ctx):
    _chk(lib().pdg_destroy(ctx), ctx)


def pdg_set_nodes(ctx, n, d_q, d_log_unary):
    _chk(lib().pdg_set_nodes(ctx, n, d_q, d_log_unary), ctx)


def pdg_insert_edges(ctx, m, d_src, d_dst, d_log_phi, d_uid_out):
    _chk(lib().pdg_insert_edges(ctx, m, d_src, d_dst, d_log_phi, d_uid_out), ctx)


def pdg_remove_edges(ctx, m, d_uid):
    _chk(lib().pdg_remove_edges(ctx, m, d_uid), ctx)


def pdg_num_edges(ctx) -> int:
    v = _I64(0)
    _chk(lib().pdg_num_edges(ctx, ctypes.byref(v)), ctx)
    return v.value


def pdg_live_uids(ctx, d_uid_out):
    _chk(lib().pdg_live_uids(ctx, d_uid_out), ctx)


def pdg_decompose(m, q_max, d_qs, d_qd, d_log_phi, precision, d_params_out, stream=0):
    _chk(lib().pdg_decompose(m, q_max, d_qs, d_qd, d_log_phi, precision, d_params_out, stream))


def pdg_params_layout(q_max):
    """(bytes per edge, offset of sign, thr, h, c0)."""
    v = [_I64(0) for _ in range(5)]
    _chk(lib().pdg_params_layout(q_max, *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


def pdg_init_chains(ctx):
    _chk(lib().pdg_init_chains(ctx), ctx)


def pdg_set_state(ctx, d_x):
    _chk(lib().pdg_set_state(ctx, d_x), ctx)


def pdg_get_state(ctx, d_x_out):
    _chk(lib().pdg_get_state(ctx, d_x_out), ctx)


def pdg_get_sweep(ctx) -> int:
    v = _I64(0)
    _chk(lib().pdg_get_sweep(ctx, ctypes.byref(v)), ctx)
    return v.value


def pdg_set_sweep(ctx, t):
    _chk(lib().pdg_set_sweep(ctx, t), ctx)


def pdg_sweep(ctx, n_sweeps):
    _chk(lib().pdg_sweep(ctx, n_sweeps), ctx)


def pdg_dual_phase(ctx):
    _chk(lib().pdg_dual_phase(ctx), ctx)


def pdg_primal_phase(ctx):
    _chk(lib().pdg_primal_phase(ctx), ctx)


def pdg_get_duals(ctx, m, d_uid, d_theta_out):
    _chk(lib().pdg_get_duals(ctx, m, d_uid, d_theta_out), ctx)


def pdg_log_v(ctx, d_out):
    _chk(lib().pdg_log_v(ctx, d_out), ctx)


def pdg_log_v_noalloc(ctx, d_out):
    _chk(lib().pdg_log_v_noalloc(ctx, d_out), ctx)


def pdg_graph_create(ctxs, n_sweeps):
    arr = (_P * len(ctxs))(*[c.value if isinstance(c, _P) else c for c in ctxs])
    out = _P()
    _chk(lib().pdg_graph_create(arr, len(ctxs), n_sweeps, ctypes.byref(out)))
    return out


def pdg_graph_launch(graph):
    _chk(lib().pdg_graph_launch(graph))


def pdg_graph_destroy(graph):
    _chk(lib().pdg_graph_destroy(graph))


def pdg_tune(ctx, reps=5) -> pdg_tuning:
    out = pdg_tuning()
    _chk(lib().pdg_tune(ctx, reps, ctypes.byref(out)), ctx)
    return out


def pdg_set_tuning(ctx, tuning: pdg_tuning):
    _chk(lib().pdg_set_tuning(ctx, ctypes.byref(tuning)), ctx)


def pdg_get_tuning(ctx) -> pdg_tuning:
    out = pdg_tuning()
    _chk(lib().pdg_get_tuning(ctx, ctypes.byref(out)), ctx)
    return out


def pdg_get_marginals(ctx, d_out) -> int:
    v = _I64(0)
    _chk(lib().pdg_get_marginals(ctx, d_out, ctypes.byref(v)), ctx)
    return v.value


def pdg_get_counts(ctx, d_out) -> int:
    v = _I64(0)
    _chk(lib().pdg_get_counts(ctx, d_out, ctypes.byref(v)), ctx)
    return v.value


def pdg_reset_marginals(ctx):
    _chk(lib().pdg_reset_marginals(ctx), ctx)


def pdg_sync(ctx):
    _chk(lib().pdg_sync(ctx), ctx)


# --------------------------------------------------------- torch convenience
class Sampler:
    """A context whose inputs live in torch device tensors.

    ``model`` is a ``workloads.Model``; its table dtype selects the precision
    (float32 -> FP32 tables and FP32 exp in the node draw, float64 -> FP64)."""

    def __init__(self, model, n_chains: int, seed: int = 0, burn_in: int = 0,
                 edge_capacity: int | None = None, device: int = 0, stream: int | None = None):
        import torch
        self.torch = torch
        self.dev = torch.device("cuda", device)
        self.n, self.C, self.q_max = model.n, n_chains, model.q_max
        self.fp64 = model.Lam.dtype == np.float64
        self.tdt = torch.float64 if self.fp64 else torch.float32
        self.stream = torch.cuda.current_stream(self.dev).cuda_stream if stream is None else stream
        cfg = pdg_config(seed=seed, n_chains=n_chains, q_max=model.q_max,
                         node_capacity=model.n,
                         edge_capacity=edge_capacity or max(model.m, 1),
                         precision=PDG_PRECISION_F64 if self.fp64 else PDG_PRECISION_F32,
                         reserved=0, burn_in=burn_in)
        self.ctx = pdg_create(cfg, device, self.stream)
        q = torch.as_tensor(np.asarray(model.q, np.int32), device=self.dev)
        lam = torch.as_tensor(np.ascontiguousarray(model.lam), device=self.dev).to(self.tdt)
        pdg_set_nodes(self.ctx, self.n, q.data_ptr(), lam.data_ptr())
        self.uids = self.insert_edges(model.src, model.dst, model.Lam) if model.m else \
            torch.zeros(0, dtype=torch.int64, device=self.dev)

    def close(self):
        if self.ctx is not None:
            pdg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a, dtype):
        t = self.torch
        return t.as_tensor(np.ascontiguousarray(a), device=self.dev).to(dtype).contiguous()

    def insert_edges(self, src, dst, Lam):
        t = self.torch
        m = len(src)
        s = self._dev(np.asarray(src, np.int32), t.int32)
        d = self._dev(np.asarray(dst, np.int32), t.int32)
        L = self._dev(Lam, self.tdt)
        uid = t.zeros(m, dtype=t.int64, device=self.dev)
        pdg_insert_edges(self.ctx, m, s.data_ptr(), d.data_ptr(), L.data_ptr(), uid.data_ptr())
        return uid

    def remove_edges(self, uids):
        t = self.torch
        u = uids if isinstance(uids, t.Tensor) else self._dev(np.asarray(uids, np.uint64).view(np.int64), t.int64)
        pdg_remove_edges(self.ctx, len(u), u.data_ptr())

    def live_uids(self):
        t = self.torch
        k = pdg_num_edges(self.ctx)
        out = t.zeros(k, dtype=t.int64, device=self.dev)
        if k:
            pdg_live_uids(self.ctx, out.data_ptr())
        return out

    def init(self):
        pdg_init_chains(self.ctx)

    def sweep(self, n=1):
        pdg_sweep(self.ctx, n)

    def dual_phase(self):
        pdg_dual_phase(self.ctx)

    def primal_phase(self):
        pdg_primal_phase(self.ctx)

    def state(self):
        x = self.torch.empty((self.n, self.C), dtype=self.torch.uint8, device=self.dev)
        pdg_get_state(self.ctx, x.data_ptr())
        return x

    def set_state(self, x):
        x = x if isinstance(x, self.torch.Tensor) else self._dev(x, self.torch.uint8)
        assert x.shape == (self.n, self.C) and x.dtype == self.torch.uint8
        x = x.contiguous()
        pdg_set_state(self.ctx, x.data_ptr())
        pdg_sync(self.ctx)

    @property
    def t(self):
        return pdg_get_sweep(self.ctx)

    @t.setter
    def t(self, value):
        pdg_set_sweep(self.ctx, value)

    def duals(self, uids):
        out = self.torch.empty((len(uids), self.C), dtype=self.torch.int64, device=self.dev)
        pdg_get_duals(self.ctx, len(uids), uids.data_ptr(), out.data_ptr())
        return out

    def log_v(self):
        """log V(x, theta) per chain (float64 [C]) between the two phases of a sweep."""
        out = self.torch.empty(self.C, dtype=self.torch.float64, device=self.dev)
        pdg_log_v(self.ctx, out.data_ptr())
        return out

    def marginals(self):
        out = self.torch.empty((self.n, self.q_max), dtype=self.torch.float64, device=self.dev)
        s = pdg_get_marginals(self.ctx, out.data_ptr())
        return out, s

    def counts(self):
        """Raw counters (int64 [n][q_max] on the host) and the samples they hold."""
        out = self.torch.zeros((self.n, self.q_max), dtype=self.torch.int32, device=self.dev)
        s = pdg_get_counts(self.ctx, out.data_ptr())
        return out.cpu().numpy().view(np.uint32).astype(np.int64), s

    def reset_marginals(self):
        pdg_reset_marginals(self.ctx)

    def sync(self):
        pdg_sync(self.ctx)

"""ctypes binding of the learned block proposal (include/pdg_block.h), with the
same function names, loaded from libpdg.so.  The ``pdg_blk_*`` / ``pdg_mlp_*``
functions only marshal arguments; every step runs in the library's kernels.

``BlockProposal`` keeps the proposal network's parameters and buffers in torch
device tensors (memory and stream only) and chains the calls of one learned
step and one training step.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import pdg

_P, _I32, _I64, _F32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
S = _I32

MLP_IN, MLP_HID, MLP_OUT = 96, 256, 64
OFF = {"W1": 0, "b1": 24576, "W2": 24832, "b2": 90368, "W3": 90624, "b3": 107008}
SHAPE = {"W1": (256, 96), "b1": (256,), "W2": (256, 256), "b2": (256,), "W3": (64, 256),
         "b3": (64,)}
MLP_PARAMS = 107072

EXPORTS = ["pdg_blk_create", "pdg_blk_destroy", "pdg_blk_cut_duals", "pdg_blk_inputs",
           "pdg_blk_mh", "pdg_blk_get_cut_duals", "pdg_blk_info", "pdg_blk_set_step",
           "pdg_mlp_forward", "pdg_mlp_backward_workspace", "pdg_mlp_backward", "pdg_mlp_adam",
           "pdg_dense_fields"]

_SIG = {
    "pdg_blk_create": [_P, _I32, _I32, _P, _P, ctypes.POINTER(_P)],
    "pdg_blk_destroy": [_P],
    "pdg_blk_cut_duals": [_P],
    "pdg_blk_inputs": [_P, _P, _P, _P],
    "pdg_blk_mh": [_P, _P, _P, _P, _P],
    "pdg_blk_get_cut_duals": [_P, _P],
    "pdg_blk_info": [_P] + [ctypes.POINTER(_I64)] * 4,
    "pdg_blk_set_step": [_P, _I64],
    "pdg_mlp_forward": [_P, _P, _I64, _P, _P, _P, _P, _P],
    "pdg_mlp_backward_workspace": [_I64, ctypes.POINTER(_I64)],
    "pdg_mlp_backward": [_P, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _I64, _P],
    "pdg_mlp_adam": [_P, _P, _P, _P, _I64, _F32, _F32, _F32, _F32, _P, _P],
    "pdg_dense_fields": [_P, _I64, _P, _I32, _P],
}
_declared = False


def _lib():
    global _declared
    L = pdg.lib()
    if not _declared:
        for name, args in _SIG.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = S
        _declared = True
    return L


def _chk(code, ctx=None):
    if code != pdg.PDG_OK:
        raise pdg.PdgError(code, pdg.pdg_last_error(ctx))


def pdg_blk_create(ctx, H, W, d_log_phi, d_log_unary):
    out = _P()
    _chk(_lib().pdg_blk_create(ctx, H, W, d_log_phi, d_log_unary, ctypes.byref(out)), ctx)
    return out


def pdg_blk_destroy(blk):
    _chk(_lib().pdg_blk_destroy(blk))


def pdg_blk_cut_duals(blk, ctx=None):
    _chk(_lib().pdg_blk_cut_duals(blk), ctx)


def pdg_blk_inputs(blk, d_in, d_target=0, d_fields=0, ctx=None):
    _chk(_lib().pdg_blk_inputs(blk, d_in, d_target or None, d_fields or None), ctx)


def pdg_blk_mh(blk, d_logits, d_prop=0, d_acc=0, d_flag=0, ctx=None):
    _chk(_lib().pdg_blk_mh(blk, d_logits, d_prop or None, d_acc or None, d_flag or None), ctx)


def pdg_blk_get_cut_duals(blk, d_theta, ctx=None):
    _chk(_lib().pdg_blk_get_cut_duals(blk, d_theta), ctx)


def pdg_blk_info(blk, ctx=None):
    v = [_I64(0) for _ in range(4)]
    _chk(_lib().pdg_blk_info(blk, *[ctypes.byref(a) for a in v]), ctx)
    return tuple(a.value for a in v)


def pdg_blk_set_step(blk, s, ctx=None):
    _chk(_lib().pdg_blk_set_step(blk, s), ctx)


def pdg_mlp_forward(d_wbf, d_w32, rows, d_in, d_logits, d_h1=0, d_h2=0, stream=0):
    _chk(_lib().pdg_mlp_forward(d_wbf, d_w32, rows, d_in, d_logits, d_h1 or None, d_h2 or None,
                                stream))


def pdg_mlp_backward_workspace(rows) -> int:
    v = _I64(0)
    _chk(_lib().pdg_mlp_backward_workspace(rows, ctypes.byref(v)))
    return v.value


def pdg_mlp_backward(d_wbf, rows, d_in, d_h1, d_h2, d_logits, d_target, d_grad, d_loss, d_work,
                     work_bytes, stream=0):
    _chk(_lib().pdg_mlp_backward(d_wbf, rows, d_in, d_h1, d_h2, d_logits, d_target, d_grad,
                                 d_loss or None, d_work, work_bytes, stream))


def pdg_mlp_adam(d_w, d_g, d_m, d_v, step, lr, beta1, beta2, eps, d_wbf, stream=0):
    _chk(_lib().pdg_mlp_adam(d_w, d_g, d_m, d_v, step, lr, beta1, beta2, eps, d_wbf, stream))


def pdg_dense_fields(ctx, n, d_nodes, method, d_out):
    _chk(_lib().pdg_dense_fields(ctx, n, d_nodes, method, d_out), ctx)


def bf16_bits(a: np.ndarray) -> np.ndarray:
    """float array -> bfloat16 bit patterns (uint16), round to nearest even; the
    host side of parameter initialisation (the device keeps its own copy in
    step with pdg_mlp_adam)."""
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


class BlockProposal:
    """Learned proposal for the 8x8 blocks of a binary grid sampler.

    sampler: a ``pdg.Sampler`` over the grid model (binary, n = H W); the block
    object reads the same tables.  Parameters are initialised with
    He-scaled normal weights (seeded) and zero biases."""

    def __init__(self, sampler, model, H, W, init_seed=0, batch_rows=8192):
        import torch
        self.t = torch
        self.s, self.dev = sampler, sampler.dev
        self.stream = sampler.stream
        self.H, self.W = H, W
        Lam = torch.as_tensor(np.ascontiguousarray(model.Lam), device=self.dev).to(sampler.tdt)
        lam = torch.as_tensor(np.ascontiguousarray(model.lam), device=self.dev).to(sampler.tdt)
        self.blk = pdg_blk_create(sampler.ctx, H, W, Lam.data_ptr(), lam.data_ptr())
        _, self.nb, _, _ = pdg_blk_info(self.blk, sampler.ctx)
        self.rows = self.nb * sampler.C
        rng = np.random.default_rng(init_seed)
        w = np.zeros(MLP_PARAMS, np.float32)
        for name, shp in SHAPE.items():
            if name.startswith("W"):
                std = np.sqrt(2.0 / shp[1]) * (0.1 if name == "W3" else 1.0)
                w[OFF[name]:OFF[name] + int(np.prod(shp))] = rng.normal(0, std, size=shp).ravel()
        self.w32 = torch.as_tensor(w, device=self.dev)
        self.wbf = torch.as_tensor(bf16_bits(w).view(np.int16), device=self.dev)
        self.m = torch.zeros_like(self.w32)
        self.v = torch.zeros_like(self.w32)
        self.g = torch.zeros_like(self.w32)
        self.step_count = 0
        self.x_in = torch.zeros((self.rows, MLP_IN), dtype=torch.int16, device=self.dev)
        self.logits = torch.zeros((self.rows, MLP_OUT), dtype=torch.float32, device=self.dev)
        self.batch_rows = batch_rows
        self.loss = torch.zeros(1, dtype=torch.float64, device=self.dev)

    def close(self):
        if self.blk is not None:
            pdg_blk_destroy(self.blk)
            self.blk = None

    def set_params(self, w: np.ndarray):
        """Packed FP32 parameters (the BF16 copy follows by rounding)."""
        w = np.ascontiguousarray(w, np.float32)
        self.w32.copy_(self.t.as_tensor(w, device=self.dev))
        self.wbf.copy_(self.t.as_tensor(bf16_bits(w).view(np.int16), device=self.dev))

    # ---- one learned step: cut duals, inputs, network, MH
    def step(self, prop=None, acc=None, flag=None, fields=None, target=None):
        ctx = self.s.ctx
        pdg_blk_cut_duals(self.blk, ctx)
        pdg_blk_inputs(self.blk, self.x_in.data_ptr(), target.data_ptr() if target is not None else 0,
                       fields.data_ptr() if fields is not None else 0, ctx)
        pdg_mlp_forward(self.wbf.data_ptr(), self.w32.data_ptr(), self.rows, self.x_in.data_ptr(),
                        self.logits.data_ptr(), stream=self.stream)
        pdg_blk_mh(self.blk, self.logits.data_ptr(), prop.data_ptr() if prop is not None else 0,
                   acc.data_ptr() if acc is not None else 0,
                   flag.data_ptr() if flag is not None else 0, ctx)

    def sample_training_rows(self, x_out, t_out):
        """Cut duals from the sampler's current state and the resulting input rows
        and targets (the block states), into x_out [rows][96] / t_out [rows][64]."""
        ctx = self.s.ctx
        pdg_blk_cut_duals(self.blk, ctx)
        pdg_blk_inputs(self.blk, x_out.data_ptr(), t_out.data_ptr(), 0, ctx)

    # ---- one Adam step on a batch of training rows
    def train_step(self, X, T, lr=1e-3):
        t = self.t
        R = X.shape[0]
        if not hasattr(self, "_h1") or self._h1.shape[0] < R:
            self._h1 = t.empty((R, MLP_HID), dtype=t.int16, device=self.dev)
            self._h2 = t.empty((R, MLP_HID), dtype=t.int16, device=self.dev)
            self._lg = t.empty((R, MLP_OUT), dtype=t.float32, device=self.dev)
            nbytes = pdg_mlp_backward_workspace(R)
            self._work = t.empty(nbytes, dtype=t.uint8, device=self.dev)
        pdg_mlp_forward(self.wbf.data_ptr(), self.w32.data_ptr(), R, X.data_ptr(),
                        self._lg.data_ptr(), self._h1.data_ptr(), self._h2.data_ptr(), self.stream)
        pdg_mlp_backward(self.wbf.data_ptr(), R, X.data_ptr(), self._h1.data_ptr(),
                         self._h2.data_ptr(), self._lg.data_ptr(), T.data_ptr(),
                         self.g.data_ptr(), self.loss.data_ptr(), self._work.data_ptr(),
                         self._work.numel(), self.stream)
        self.step_count += 1
        pdg_mlp_adam(self.w32.data_ptr(), self.g.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
                     self.step_count, lr, 0.9, 0.999, 1e-8, self.wbf.data_ptr(), self.stream)

    def accept_rate(self):
        s, nb, acc, prop = pdg_blk_info(self.blk, self.s.ctx)
        return acc / max(prop, 1)

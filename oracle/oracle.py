"""ctypes front-end of the FP64 CPU oracle (``pdg_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``.  The GPU library never loads it.

Every function here only marshals numpy arrays; the arithmetic is in the C file,
whose header maps each function to the passage of the paper it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "pdg_oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")

PHASE_INIT, PHASE_DUAL, PHASE_PRIMAL = 0, 1, 2

_lib = None


LIB_NATIVE = os.path.join(_HERE, "liboracle_native.so")
FLAGS = ["-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off"]
# for timing on the host it runs on (CPU baseline): same source and arithmetic
# (no contraction into FMA), tuned for that host's instruction set
FLAGS_NATIVE = ["-O3", "-march=native", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                "-ffp-contract=off"]


def build() -> str:
    """Compile the oracle with gcc (portable -O2, OpenMP over chains)."""
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", *FLAGS, "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"])
    os.replace(tmp, LIB)
    return LIB


def build_native() -> str:
    """Compile a copy for this host's CPU (-O3 -march=native) and return its path;
    load it with use_library()."""
    tmp = LIB_NATIVE + ".tmp"
    subprocess.check_call(["gcc", *FLAGS_NATIVE, "-o", tmp, SRC, "-lm"])
    os.replace(tmp, LIB_NATIVE)
    return LIB_NATIVE


def use_library(path):
    """Point the wrappers at another build of the oracle (the mutation tests load
    deliberately broken copies); ``None`` returns to the default build."""
    global _lib
    if path is None:
        _lib = None
        return
    _lib = ctypes.CDLL(path)
    _declare(_lib)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = ctypes.CDLL(LIB)
        _declare(_lib)
    return _lib


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_U64 = ctypes.c_uint64
_U32 = ctypes.c_uint32


def _declare(L):
    L.orc_philox4x32_10.argtypes = [_P, _P, _P]
    L.orc_philox4x32_10.restype = None
    L.orc_uniform.argtypes = [_U64, _U32, _U64, _U32, _U32, ctypes.c_int]
    L.orc_uniform.restype = ctypes.c_double
    L.orc_factor2x2.argtypes = [_P, _P, _P]
    L.orc_factor2x2.restype = None
    L.orc_theorem_params.argtypes = [_P, _P, _P]
    L.orc_theorem_params.restype = None
    L.orc_decompose.argtypes = [_I64, _I32, _P, _P, _P, _P, _P, _P]
    L.orc_decompose.restype = ctypes.c_int
    L.orc_dual_p1.argtypes = [_P, ctypes.c_int, ctypes.c_int]
    L.orc_dual_p1.restype = ctypes.c_double
    L.orc_init.argtypes = [_I64, _I32, _P, _U64, _P]
    L.orc_init.restype = None
    L.orc_dual_edge.argtypes = [_I32, _I32, _I32, _P, _I32, _I32, _U64, _I32, _U32, _U64,
                                _P, _P]
    L.orc_dual_edge.restype = None
    L.orc_node_logits.argtypes = [_I32, _I32, _P, _I64, _P, _P, _P, _P, _P, _P]
    L.orc_node_logits.restype = None
    L.orc_primal_node.argtypes = [_I32, _I32, _P, _I64, _P, _P, _P, _P, _P, _I64, _I32,
                                  _U32, _U64, _P, _P]
    L.orc_primal_node.restype = None
    L.orc_sweep.argtypes = [_I64, _I64, _I32, _I32, _P, _P, _P, _P, _P, _P, _P, _P, _U64,
                            _U32, _P, _P, _P, _P, _P]
    L.orc_sweep.restype = ctypes.c_int
    L.orc_run.argtypes = [_I64, _I64, _I32, _I32, _P, _P, _P, _P, _P, _P, _P, _P, _U64,
                          _U32, _I64, _I64, _P, _P, _P, _P]
    L.orc_run.restype = ctypes.c_int
    L.orc_primal_phase.argtypes = [_I64, _I64, _I32, _I32, _P, _P, _P, _P, _P, _P, _P, _U64,
                                   _U32, _P, _P, _P]
    L.orc_primal_phase.restype = ctypes.c_int
    L.orc_num_threads.argtypes = []
    L.orc_num_threads.restype = ctypes.c_int
    L.orc_uniform_batch.argtypes = [_U64, _U32, _U32, _I64, _P, _P, _P, _P]
    L.orc_uniform_batch.restype = None
    L.orc_set_threads.argtypes = [_I32]
    L.orc_set_threads.restype = None
    L.orc_all_logits.argtypes = [_I64, _I64, _I32, _P, _P, _P, _P, _P, _P, _P, _P, _P]
    L.orc_all_logits.restype = ctypes.c_int
    L.orc_log_v.argtypes = [_I64, _I64, _I32, _I32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                            _P]
    L.orc_log_v.restype = ctypes.c_int
    L.orc_dual_decide.argtypes = [_P, _I32, _I32, ctypes.c_double, _P]
    L.orc_dual_decide.restype = ctypes.c_int
    L.orc_categorical_draw.argtypes = [_I32, _P, ctypes.c_double, _P]
    L.orc_categorical_draw.restype = _I32


def _c(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(_P)


# --------------------------------------------------------------------------- RNG
def philox4x32_10(ctr, key) -> np.ndarray:
    c, pc = _c(ctr, np.uint32)
    k, pk = _c(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(pc, pk, out.ctypes.data_as(_P))
    return out


def uniform(seed, phase, ident, sub, sweep, slot) -> float:
    return lib().orc_uniform(seed, phase, ident, sub, sweep, slot)


def uniforms(seed, phase, sweep, ids, subs, slots) -> np.ndarray:
    """Vector form of uniform(): arrays ids (u64), subs (u32), slots (0..4)."""
    shape = np.broadcast(np.asarray(ids), np.asarray(subs), np.asarray(slots)).shape
    ids, pi = _c(np.broadcast_to(np.asarray(ids, np.uint64), shape).ravel(), np.uint64)
    subs, ps = _c(np.broadcast_to(subs, shape).ravel(), np.uint32)
    slots, pl = _c(np.broadcast_to(slots, shape).ravel(), np.int32)
    out = np.zeros(shape, np.float64)
    lib().orc_uniform_batch(int(seed), int(phase), int(sweep), out.size, pi, ps, pl,
                            out.ctypes.data_as(_P))
    return out


# ----------------------------------------------------------------- decomposition
def factor2x2(P):
    P, pp = _c(np.asarray(P, np.float64).reshape(4), np.float64)
    B = np.zeros(4)
    C = np.zeros(4)
    lib().orc_factor2x2(pp, B.ctypes.data_as(_P), C.ctypes.data_as(_P))
    return B.reshape(2, 2), C.reshape(2, 2)


def theorem_params(B, C) -> np.ndarray:
    B, pb = _c(np.asarray(B).reshape(4), np.float64)
    C, pc = _c(np.asarray(C).reshape(4), np.float64)
    out = np.zeros(5)
    lib().orc_theorem_params(pb, pc, out.ctypes.data_as(_P))
    return out


def dual_p1(par5, y, yp) -> float:
    p, pp = _c(par5, np.float64)
    return lib().orc_dual_p1(pp, int(y), int(yp))


def dual_decide(par5, y, yp, u):
    """theta and flag of one dual draw with its uniform u given."""
    p, pp = _c(par5, np.float64)
    f = ctypes.c_int32(0)
    th = lib().orc_dual_decide(pp, int(y), int(yp), float(u), ctypes.byref(f))
    return int(th), int(f.value)


def categorical_draw(L, u):
    """State and flag of one node draw from logits L with its uniform u given."""
    Lc, pl = _c(L, np.float64)
    f = ctypes.c_int32(0)
    x = lib().orc_categorical_draw(len(Lc), pl, float(u), ctypes.byref(f))
    return int(x), int(f.value)


class Decomposition:
    """Per-edge parameters: par [m][(q_max-1)^2][5] = (alpha1, alpha2, q, beta1, beta2),
    rrow/rcol [m][q_max] the unary parts carried by the src/dst endpoint."""

    def __init__(self, par, rrow, rcol):
        self.par, self.rrow, self.rcol = par, rrow, rcol


def decompose(model) -> Decomposition:
    m, qm = model.m, model.q_max
    D = (qm - 1) * (qm - 1)
    qs, pqs = _c(model.q[model.src], np.int32)
    qd, pqd = _c(model.q[model.dst], np.int32)
    Lam, pL = _c(model.Lam, np.float64)
    par = np.zeros((m, max(D, 1), 5))
    rrow = np.zeros((m, qm))
    rcol = np.zeros((m, qm))
    rc = lib().orc_decompose(m, qm, pqs, pqd, pL, par.ctypes.data_as(_P),
                             rrow.ctypes.data_as(_P), rcol.ctypes.data_as(_P))
    if rc != 0:
        raise ValueError("factor table is not strictly positive (non-finite log entry)")
    return Decomposition(par, rrow, rcol)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(k: int) -> None:
    lib().orc_set_threads(int(k))


# ------------------------------------------------------------------------ sweeps
def init_state(model, C, seed) -> np.ndarray:
    q, pq = _c(model.q, np.int32)
    x = np.zeros((model.n, C), np.uint8)
    lib().orc_init(model.n, C, pq, seed, x.ctypes.data_as(_P))
    return x


def _graph_args(model, dec, uid):
    keep = []

    def p(a, dt):
        a, ptr = _c(a, dt)
        keep.append(a)
        return ptr

    args = [p(model.q, np.int32), p(model.lam, np.float64), p(model.src, np.int32),
            p(model.dst, np.int32), p(uid, np.uint64), p(dec.par, np.float64),
            p(dec.rrow, np.float64), p(dec.rcol, np.float64)]
    return args, keep


def sweep(model, dec, uid, seed, t, x_in):
    """One teacher-forced sweep t: returns (theta [m][C] u64, dflag [m][C] u64,
    x_out [n][C] u8, pflag [n][C] u8)."""
    x_in = np.ascontiguousarray(x_in, np.uint8)
    n, C = x_in.shape
    theta = np.zeros((model.m, C), np.uint64)
    dflag = np.zeros((model.m, C), np.uint64)
    x_out = np.zeros((n, C), np.uint8)
    pflag = np.zeros((n, C), np.uint8)
    args, keep = _graph_args(model, dec, uid)
    rc = lib().orc_sweep(model.n, model.m, C, model.q_max, *args, seed, t,
                         x_in.ctypes.data_as(_P), theta.ctypes.data_as(_P),
                         dflag.ctypes.data_as(_P), x_out.ctypes.data_as(_P),
                         pflag.ctypes.data_as(_P))
    if rc != 0:
        raise MemoryError("oracle sweep failed")
    return theta, dflag, x_out, pflag


def primal_phase(model, dec, seed, t, theta):
    """Primal phase of sweep t from given duals theta [m][C] (u64 bit d):
    returns (x_out [n][C] u8, pflag [n][C] u8)."""
    theta = np.ascontiguousarray(theta, np.uint64)
    C = theta.shape[1] if theta.ndim == 2 else 1
    x_out = np.zeros((model.n, C), np.uint8)
    pflag = np.zeros((model.n, C), np.uint8)
    args, keep = _graph_args(model, dec, np.zeros(model.m, np.uint64))
    a = [args[0], args[1], args[2], args[3], args[5], args[6], args[7]]
    rc = lib().orc_primal_phase(model.n, model.m, C, model.q_max, *a, seed, t,
                                theta.ctypes.data_as(_P), x_out.ctypes.data_as(_P),
                                pflag.ctypes.data_as(_P))
    if rc != 0:
        raise MemoryError("oracle primal phase failed")
    return x_out, pflag


def run(model, dec, uid, seed, x, t0, n_sweeps, burn_in, counts=None):
    """Free-running sweeps t0+1..t0+n_sweeps on x (modified in place).
    Returns (counts [n][q_max] u64, n_flagged, n_draws)."""
    assert x.dtype == np.uint8 and x.flags.c_contiguous
    C = x.shape[1]
    if counts is None:
        counts = np.zeros((model.n, model.q_max), np.uint64)
    nf = ctypes.c_int64(0)
    nd = ctypes.c_int64(0)
    args, keep = _graph_args(model, dec, uid)
    rc = lib().orc_run(model.n, model.m, C, model.q_max, *args, seed, t0, n_sweeps, burn_in,
                       x.ctypes.data_as(_P), counts.ctypes.data_as(_P), ctypes.byref(nf),
                       ctypes.byref(nd))
    if rc != 0:
        raise MemoryError("oracle run failed")
    return counts, nf.value, nd.value


def all_logits(model, dec, theta_one_chain) -> np.ndarray:
    L = np.zeros((model.n, model.q_max))
    args, keep = _graph_args(model, dec, np.zeros(model.m, np.uint64))
    th, pth = _c(theta_one_chain, np.uint64)
    a = [args[0], args[1], args[2], args[3], args[5], args[6], args[7]]
    rc = lib().orc_all_logits(model.n, model.m, model.q_max, *a, pth, L.ctypes.data_as(_P))
    if rc != 0:
        raise MemoryError("oracle logits failed")
    return L


def log_v(model, dec, theta, x) -> np.ndarray:
    """log V(x, theta) per chain (Sec. 5.2 estimator of the partition function):
    theta [m][C] u64 (bit d), x [n][C] u8 -> [C] float64."""
    theta = np.ascontiguousarray(theta, np.uint64).reshape(model.m, -1)
    x = np.ascontiguousarray(x, np.uint8).reshape(model.n, -1)
    C = x.shape[1]
    out = np.zeros(C)
    args, keep = _graph_args(model, dec, np.zeros(model.m, np.uint64))
    Lam, pL = _c(model.Lam, np.float64)
    a = [args[0], args[1], args[2], args[3], pL, args[5], args[6], args[7]]
    rc = lib().orc_log_v(model.n, model.m, C, model.q_max, *a, theta.ctypes.data_as(_P),
                         x.ctypes.data_as(_P), out.ctypes.data_as(_P))
    if rc != 0:
        raise MemoryError("oracle log V failed")
    return out


# --------------------------------------------------- single elements (sampled checks)
def dual_edge(model, dec, e, x_src, x_dst, uid_e, c, t, seed):
    """theta bits and flag bits (u64, bit d) of edge e for chain c at sweep t."""
    qm = model.q_max
    par, pp = _c(dec.par[e], np.float64)
    th = ctypes.c_uint64(0)
    fl = ctypes.c_uint64(0)
    lib().orc_dual_edge(int(model.q[model.src[e]]), int(model.q[model.dst[e]]), qm, pp,
                        int(x_src), int(x_dst), int(uid_e), int(c), int(t), int(seed),
                        ctypes.byref(th), ctypes.byref(fl))
    return th.value, fl.value


def primal_node(model, dec, i, inc_edges, inc_sides, inc_theta, c, t, seed):
    """x and flag of node i for chain c at sweep t, given the duals of its incident
    edges (inc_edges: edge rows of the model, inc_sides: 0 = node is src, 1 = dst)."""
    inc_edges = np.asarray(inc_edges, np.int64)
    inc_sides = np.asarray(inc_sides, np.int32)
    k = len(inc_edges)
    qother = np.where(inc_sides == 0, model.q[model.dst[inc_edges]],
                      model.q[model.src[inc_edges]]).astype(np.int32)
    par = np.ascontiguousarray(dec.par[inc_edges])
    r = np.ascontiguousarray(np.where(inc_sides[:, None] == 0, dec.rrow[inc_edges],
                                      dec.rcol[inc_edges]))
    lam, pl = _c(model.lam[i], np.float64)
    sd, psd = _c(inc_sides, np.int32)
    qo, pqo = _c(qother, np.int32)
    pa, ppa = _c(par, np.float64)
    rr, prr = _c(r, np.float64)
    th, pth = _c(np.asarray(inc_theta, np.uint64), np.uint64)
    xo = ctypes.c_int32(0)
    fo = ctypes.c_int32(0)
    lib().orc_primal_node(int(model.q[i]), model.q_max, pl, k, psd, pqo, ppa, prr, pth,
                          int(i), int(c), int(t), int(seed), ctypes.byref(xo),
                          ctypes.byref(fo))
    return xo.value, fo.value

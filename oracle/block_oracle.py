"""FP64 oracle of the learned block proposal (blocking of Sec. 5.4).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and by the benchmark's CPU
baseline.  It shares no code with the GPU library; generator values come from
the C oracle (``oracle.py``), the decomposition of the cut edges' tables too.

Blocking (Sec. 5.4): the duals are split into theta_1, here the duals of the
edges that cross block boundaries ("cut" edges), and theta_0, the rest.  Given
theta_1 the blocks are independent: with the Lemma of Sec. 3,
p(x, theta_1) is proportional to prod_i u_i prod_{internal e} phi_e
prod_{cut e} w(theta_e) g_e(x_src, theta_e) h_e(x_dst, theta_e), so
p(x_B | theta_1) for a binary block B is proportional to
exp(sum_i f_i x_i + sum_{internal e} l_e x_src x_dst) with
  f_i = log u_i(1) - log u_i(0)
        + sum_{internal e, i src} (Lam_e(1,0) - Lam_e(0,0))
        + sum_{internal e, i dst} (Lam_e(0,1) - Lam_e(0,0))
        + sum_{cut e, i src} (field of state 1 of the src end given theta_e)
        + sum_{cut e, i dst} (field of state 1 of the dst end given theta_e),
  l_e = Lam_e(1,1) + Lam_e(0,0) - Lam_e(1,0) - Lam_e(0,1),
the cut-edge fields being the Theorem's alpha + theta beta plus the rescaling
unary of the one-hot decomposition (Sec. 4.1, 4.2), as in the primal phase.

One learned step s (a Metropolis-Hastings move per block, Sec. 5.4 sampling
with p(x | theta_1) replaced by an independence proposal):
  1. theta_e ~ p(theta_e | x) for every cut edge (logistic draw of Sec. 4);
  2. per block and chain, the proposal network maps the block's fields f and
     its boundary dual bits to 64 logits l; x'_i ~ Bernoulli(sigmoid(l_i));
  3. accept x'_B with probability min(1, a),
     log a = log p~(x'_B) - log p~(x_B) + log q(x_B) - log q(x'_B)
           = sum_i (x'_i - x_i)(f_i - l_i) + sum_e l_e (x'_src x'_dst - x_src x_dst).
The chain then runs the plain sweep of Sec. 5.1 (the fallback); both moves
leave p(x) invariant.

Generator (Philox4x32-10, phase 3): cut edge e (index in the grid's edge order)
draws with id 2^63 + e, sub 16 c, slot 0; block b draws its 65 uniforms with
id b, sub 16 c + floor(d / 5), slot d mod 5 (d < 64: the proposal bit of block
node d, row-major in the block; d = 64: the acceptance), all at counter s.
Flags: a draw whose uniform is within 1e-6 of p(theta = 0) (cut duals, as in
the dual phase) or of sigmoid(l) (proposal bits: the GPU evaluates the sigmoid
in FP32), or whose log u is within 1e-9 of log a (acceptance, FP64 on both
sides).

The proposal network (an MLP, BF16 weights, FP32 accumulation on the GPU) is
evaluated here in FP64 on the same BF16 values, with every activation rounded
to BF16 where the GPU rounds it (round to nearest, ties to even).
"""
from __future__ import annotations

import numpy as np

from . import oracle as O

PHASE_BLOCK = 3
CUT_ID = np.uint64(1) << np.uint64(63)
BAND_DUAL = 1e-6
BAND_PROP = 1e-6
BAND_MH = 1e-9


# ------------------------------------------------------------------ structure
class Blocking:
    """H x W grid (workloads.grid_edges numbering) cut into bs x bs blocks."""

    def __init__(self, H, W, bs):
        assert H % bs == 0 and W % bs == 0
        self.H, self.W, self.bs = H, W, bs
        self.nbr, self.nbc = H // bs, W // bs
        self.nb = self.nbr * self.nbc
        nh = H * (W - 1)
        # nodes of block b, row-major inside the block
        self.nodes = np.zeros((self.nb, bs * bs), np.int64)
        for b in range(self.nb):
            R0, C0 = (b // self.nbc) * bs, (b % self.nbc) * bs
            for p in range(bs * bs):
                self.nodes[b, p] = (R0 + p // bs) * W + C0 + p % bs
        self.block_of = np.zeros(H * W, np.int64)
        self.pos_of = np.zeros(H * W, np.int64)
        for b in range(self.nb):
            self.block_of[self.nodes[b]] = b
            self.pos_of[self.nodes[b]] = np.arange(bs * bs)
        self.h_edge = lambda r, c: r * (W - 1) + c          # (r,c)-(r,c+1)
        self.v_edge = lambda r, c: nh + r * W + c           # (r,c)-(r+1,c)
        src, dst = [], []
        for r in range(H):
            for c in range(W - 1):
                src.append(r * W + c); dst.append(r * W + c + 1)
        for r in range(H - 1):
            for c in range(W):
                src.append(r * W + c); dst.append((r + 1) * W + c)
        self.src, self.dst = np.array(src), np.array(dst)
        self.cut = self.block_of[self.src] != self.block_of[self.dst]
        # boundary bits of a block: top, bottom, left, right sides, bs each (-1 = none)
        self.bits = -np.ones((self.nb, 4 * bs), np.int64)
        for b in range(self.nb):
            R0, C0 = (b // self.nbc) * bs, (b % self.nbc) * bs
            for k in range(bs):
                if R0 > 0:
                    self.bits[b, k] = self.v_edge(R0 - 1, C0 + k)
                if R0 + bs < H:
                    self.bits[b, bs + k] = self.v_edge(R0 + bs - 1, C0 + k)
                if C0 > 0:
                    self.bits[b, 2 * bs + k] = self.h_edge(R0 + k, C0 - 1)
                if C0 + bs < W:
                    self.bits[b, 3 * bs + k] = self.h_edge(R0 + k, C0 + bs - 1)


# ------------------------------------------------------------------ conditional
def block_fields(model, dec, blk: Blocking, theta_cut):
    """f [nb][C][bs^2] and the internal couplings: (edge list of (b, p_src, p_dst),
    l_e).  theta_cut: [m][C] 0/1 for the cut edges (other rows ignored)."""
    lam = np.asarray(model.lam, np.float64)
    Lam = np.asarray(model.Lam, np.float64)
    C = theta_cut.shape[1]
    f_node = np.repeat((lam[:, 1] - lam[:, 0])[:, None], C, axis=1)  # [n][C]
    internal = []
    for e in range(model.m):
        i, j = int(model.src[e]), int(model.dst[e])
        if blk.cut[e]:
            th = theta_cut[e].astype(np.float64)
            a1, a2, _, b1, b2 = dec.par[e, 0]
            f_node[i] += dec.rrow[e, 1] + a1 + th * b1
            f_node[j] += dec.rcol[e, 1] + a2 + th * b2
        else:
            f_node[i] += Lam[e, 1, 0] - Lam[e, 0, 0]
            f_node[j] += Lam[e, 0, 1] - Lam[e, 0, 0]
            internal.append((int(blk.block_of[i]), int(blk.pos_of[i]), int(blk.pos_of[j]),
                             Lam[e, 1, 1] + Lam[e, 0, 0] - Lam[e, 1, 0] - Lam[e, 0, 1]))
    f = np.transpose(f_node[blk.nodes], (0, 2, 1))  # [nb][C][bs^2]
    return f, internal


def block_couplings(blk: Blocking, internal):
    """Dense symmetric-free form: K [nb][bs^2][bs^2] with K[b][p][q] = l_e for the
    internal edge p -> q of block b (upper entries only, as listed)."""
    k = blk.bs * blk.bs
    K = np.zeros((blk.nb, k, k))
    for b, p, q, l in internal:
        K[b, p, q] += l
    return K


def log_ptilde(xb, f, K):
    """log p~(x_B) = sum f x + x^T K x for 0/1 vectors (any leading shape)."""
    xb = np.asarray(xb, np.float64)
    return (f * xb).sum(-1) + np.einsum("...p,pq,...q->...", xb, K, xb)


# ------------------------------------------------------------------ draws
def cut_duals(model, dec, blk: Blocking, x, seed, s):
    """theta [m][C] (0 on internal edges) and flags, drawn from x at step s."""
    C = x.shape[1]
    m = model.m
    theta = np.zeros((m, C), np.uint8)
    flag = np.zeros((m, C), np.uint8)
    cut = np.flatnonzero(blk.cut)
    c = np.arange(C, dtype=np.uint32)
    ids = (CUT_ID | cut.astype(np.uint64))[:, None]
    u = O.uniforms(seed, PHASE_BLOCK, s, np.broadcast_to(ids, (len(cut), C)),
                   np.broadcast_to(16 * c[None, :], (len(cut), C)), 0)
    for k, e in enumerate(cut):
        par = dec.par[e, 0]
        y = x[model.src[e]].astype(np.float64)
        yp = x[model.dst[e]].astype(np.float64)
        p0 = 1.0 / (1.0 + np.exp(par[2] + par[3] * y + par[4] * yp))
        theta[e] = (~(u[k] < p0)).astype(np.uint8)
        flag[e] = (np.abs(u[k] - p0) < BAND_DUAL).astype(np.uint8)
    return theta, flag


def mh_log_accept(xb, xpb, f, K, logits):
    """log a of moving x_B -> x'_B under the independence proposal with logits."""
    return log_ptilde(xpb, f, K) - log_ptilde(xb, f, K) + \
        ((np.asarray(xb, float) - np.asarray(xpb, float)) * logits).sum(-1)


def proposal_logprob(xb, logits):
    """log q(x_B) = sum_i [x_i l_i - softplus(l_i)]."""
    xb = np.asarray(xb, np.float64)
    return (xb * logits - np.logaddexp(0.0, logits)).sum(-1)


def mh_step(blk: Blocking, x, f, K, logits, seed, s, blocks=None):
    """Proposal draws and acceptance for every block (or the listed blocks,
    whose rows f, K, logits then hold in that order) and chain: returns (x_new,
    accepted [nb][C], flag [nb][C], proposals [nb][C][bs^2]).  logits (FP32
    values) [nb][C][bs^2]."""
    x_new = x.copy()
    nb, C, k = f.shape
    ids = np.arange(nb) if blocks is None else np.asarray(blocks)
    calls = (k + 1 + 4) // 5
    b_ids = ids.astype(np.uint64)[:, None, None]
    c_ids = np.arange(C, dtype=np.uint32)[None, :, None]
    d = np.arange(k + 1)[None, None, :]
    u = O.uniforms(seed, PHASE_BLOCK, s, np.broadcast_to(b_ids, (nb, C, k + 1)),
                   np.broadcast_to(16 * c_ids + (d // 5).astype(np.uint32), (nb, C, k + 1)),
                   np.broadcast_to(d % 5, (nb, C, k + 1)))
    assert calls <= 16
    lg = np.asarray(logits, np.float64)
    p1 = 1.0 / (1.0 + np.exp(-lg))
    xp = (u[..., :k] < p1).astype(np.uint8)
    flag = (np.abs(u[..., :k] - p1) < BAND_PROP).any(-1)
    xb = np.transpose(x[blk.nodes[ids]], (0, 2, 1))  # [nb][C][k]
    accepted = np.zeros((nb, C), bool)
    for b in range(nb):
        la = mh_log_accept(xb[b], xp[b], f[b], K[b], lg[b])
        lu = np.log(u[b, :, k])
        accepted[b] = lu < la
        flag[b] |= np.abs(lu - la) < BAND_MH
        for c in np.flatnonzero(accepted[b]):
            x_new[blk.nodes[ids[b]], c] = xp[b, c]
    return x_new, accepted, flag, xp


# ------------------------------------------------------------------ network
def bf16(a):
    """Round to the nearest bfloat16 value (ties to even), returned as float64."""
    f = np.asarray(a, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def mlp_inputs(blk: Blocking, f, theta_cut):
    """Network input rows [nb * C][bs^2 + 4 bs] (block-major, chain minor):
    the block's fields, then its boundary dual bits (top, bottom, left, right;
    0 where the grid has no edge), rounded to bfloat16."""
    nb, C, k = f.shape
    bits = np.zeros((nb, C, 4 * blk.bs))
    for b in range(nb):
        for t, e in enumerate(blk.bits[b]):
            if e >= 0:
                bits[b, :, t] = theta_cut[e]
    return bf16(np.concatenate([f, bits], axis=-1).reshape(nb * C, -1))


def mlp_forward(P, X, rounding=True):
    """P: dict W1 [h1][in], b1, W2 [h2][h1], b2, W3 [out][h2], b3 (BF16 weight
    values, FP32 biases).  Returns (H1, H2, logits); logits include the
    residual X[:, :out] (the block's fields)."""
    r = bf16 if rounding else (lambda a: a)
    H1 = r(np.maximum(X @ P["W1"].T + P["b1"], 0.0))
    H2 = r(np.maximum(H1 @ P["W2"].T + P["b2"], 0.0))
    out = P["W3"].shape[0]
    L = H2 @ P["W3"].T + P["b3"] + X[:, :out]
    return H1, H2, L


def mlp_loss(L, T):
    """Mean over rows of the Bernoulli negative log-likelihood of targets T."""
    return float((np.logaddexp(0.0, L) - T * L).sum(-1).mean())


def mlp_backward(P, X, H1, H2, L, T, rounding=True):
    """Gradients of mlp_loss (the residual carries no parameter), with the
    GPU's roundings of the back-propagated matrices to BF16 mirrored."""
    r = bf16 if rounding else (lambda a: a)
    R = X.shape[0]
    dl = (1.0 / (1.0 + np.exp(-L)) - T) / R
    dL = r(dl)
    g = {"W3": dL.T @ H2, "b3": dL.sum(0)}
    dH2 = r((dL @ P["W3"]) * (H2 > 0))
    g["W2"], g["b2"] = dH2.T @ H1, dH2.sum(0)
    dH1 = r((dH2 @ P["W2"]) * (H1 > 0))
    g["W1"], g["b1"] = dH1.T @ X, dH1.sum(0)
    return g


def adam(w, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba), bias-corrected; returns (w, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v

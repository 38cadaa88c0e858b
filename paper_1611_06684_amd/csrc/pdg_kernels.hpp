// HIP kernels of the primal-dual Gibbs sweep for gfx950 (wave64).
//
// Work mapping.  A wave covers P = 64 / LPI items (edges in the dual phase,
// nodes in the primal phase) times LPI chains; lane = (item, chain).  With 64
// or more chains (LPI = 64) an item owns whole waves, so everything per item
// (endpoints, parameter block, incidence segment) is wave-uniform and comes
// through scalar loads; only x, the dual bits and the draws are per lane.
//
// Storage (device, all written by this library):
//   x       uint8  [n][C]                 node states, chain fastest
//   params  block  [slot]                 per-edge decomposition (layout below)
//   z       uint32 [slot][D][Wz]          dual bit-planes: bit (c mod 32) of
//                                         word c / 32 is theta of chain c
//   inc     uint32 pool                   per-node incidence segments
//                                         [off, off + cnt): slot << 1 | side
//                                         (side 0: node is src), or kTomb
//   counts  uint32 [n][QM]                marginal counters
// Parameter block of an edge (QM = q_max, D = (QM-1)^2):
//   thr  uint64 [D]      dual thresholds (see k_decompose)
//   v    double [D]      sigma * t per entry
//   c    double [2][QM-1] constant field per state >= 1, src side then dst side
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "pdg_rng.hpp"

namespace pdg {

constexpr uint32_t kTomb = 0xFFFFFFFFu;

__host__ __device__ constexpr int dim_d(int qm) { return (qm - 1) * (qm - 1); }
__host__ __device__ constexpr int64_t block_bytes(int qm)
{
    return 16 * (int64_t)dim_d(qm) + 16 * (int64_t)(qm - 1);
}

struct Graph {
    const uint8_t *__restrict__ q;        // [n] states per node
    const double *__restrict__ lam;       // [n][QM] log unaries (FP64)
    const int32_t *__restrict__ src;      // [slots]
    const int32_t *__restrict__ dst;      // [slots]
    const uint64_t *__restrict__ uid;     // [slots], 0 = free slot
    const uint8_t *__restrict__ sq;       // [slots] q_src | q_dst << 4
    const uint8_t *__restrict__ params;   // [slots] parameter blocks
    uint32_t *__restrict__ z;             // [slots][D][Wz]
    const uint32_t *__restrict__ inc_off; // [n]
    const uint32_t *__restrict__ inc_cnt; // [n]
    const uint32_t *__restrict__ inc;     // pool
    uint8_t *__restrict__ x;              // [n][C]
    uint32_t *__restrict__ counts;        // [n][QM]
    int64_t n;
    int64_t hwm;                          // slots [0, hwm) may be live
    int32_t C;
    int32_t Wz;
    uint32_t k0, k1;                      // generator key
};

// ---------------------------------------------------------------------------
// a1: decomposition of one edge table (Sec. 4.1 + 4.2, closed form).
// For entry (a,b), a,b >= 1: ell = L(a,b) + L(0,0) - L(a,0) - L(0,b) is the
// log odds ratio of the entry's 2x2 table [[1,1],[1,e^ell]].  With
// x = |ell| / 4 and rho = sqrt(tanh x), the Remark gives tan(phi) =
// (1 - rho) / (1 + rho), so
//   t = log tan(phi) = log 2 - 2x - log1p(e^(-2x)) - 2 log1p(rho)   (<= 0),
// a form that stays finite for any finite ell.  sigma = sign(ell) records the
// row swap of the negative-determinant case.  The dual conditional is
// logistic(t k) with k = sigma(1 - 2y) + (1 - 2y') in {-2, 0, 2}, so
// p(theta = 0) = 1 / (1 + e^(t k)) takes three values and the draw compares
// the 24-bit integer U of its uniform u = (U + 0.5) 2^-24 against
// T = ceil(p0 2^24 - 0.5): theta = 0 iff U < T.  T(0) = 2^23.
// Field of the one-hot bit: src side 1/2 ell + sigma t (1 - 2 theta),
// dst side 1/2 ell + t (1 - 2 theta); the 1/2 ell and the rescaling unaries
// L(a,0) - L(0,0), L(0,b) - L(0,0) are summed into c.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double log_tan_phi(double ell)
{
    const double x = 0.25 * fabs(ell);
    const double rho = sqrt(tanh(x));
    return 0.69314718055994530942 - 2.0 * x - log1p(exp(-2.0 * x)) - 2.0 * log1p(rho);
}

__device__ __forceinline__ uint32_t threshold24(double p0)
{
    double y = ceil(p0 * 16777216.0 - 0.5);
    y = fmin(fmax(y, 0.0), 16777216.0);
    return (uint32_t)y;
}

// One thread per edge.  Reads table k (layout [m][QM][QM], type T) with node
// states qs[k], qd[k]; writes the parameter block to out + dest[k] (dest may
// be null: identity).  Sets *bad = 1 if a used entry is not finite.
template <int QM, typename T>
__global__ void k_decompose(int64_t m, const int32_t *__restrict__ qs_arr,
                            const int32_t *__restrict__ qd_arr, const T *__restrict__ phi,
                            const int32_t *__restrict__ dest, uint8_t *__restrict__ out,
                            uint32_t *__restrict__ bad)
{
    constexpr int D = dim_d(QM);
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const int qs = qs_arr[k], qd = qd_arr[k];
    if (qs < 2 || qs > QM || qd < 2 || qd > QM) {
        atomicOr(bad, 2u);
        return;
    }
    const T *L = phi + k * QM * QM;
    uint8_t *blk = out + (dest ? (int64_t)dest[k] : k) * block_bytes(QM);
    uint64_t *thr = reinterpret_cast<uint64_t *>(blk);
    double *v = reinterpret_cast<double *>(blk + 8 * D);
    double *c = reinterpret_cast<double *>(blk + 16 * D);
    int finite = 1;
    for (int a = 0; a < qs; ++a)
        for (int b = 0; b < qd; ++b) finite &= isfinite((double)L[a * QM + b]) ? 1 : 0;
    if (!finite) {
        atomicOr(bad, 1u);
        return;
    }
    const double L00 = (double)L[0];
    double crow[QM], ccol[QM];
    for (int a = 0; a < QM; ++a) crow[a] = ccol[a] = 0.0;
    for (int a = 1; a < qs; ++a) crow[a] = (double)L[a * QM] - L00;
    for (int b = 1; b < qd; ++b) ccol[b] = (double)L[b] - L00;
    for (int d = 0; d < D; ++d) {
        thr[d] = 0;
        v[d] = 0.0;
    }
    for (int a = 1; a < qs; ++a) {
        for (int b = 1; b < qd; ++b) {
            const double ell = (double)L[a * QM + b] + L00 - (double)L[a * QM] - (double)L[b];
            const double t = log_tan_phi(ell);
            const bool neg = ell < 0.0;
            const uint32_t tp = threshold24(1.0 / (1.0 + exp(2.0 * t)));
            const uint32_t tm = threshold24(1.0 / (1.0 + exp(-2.0 * t)));
            const int d = (a - 1) * (qd - 1) + (b - 1);
            thr[d] = (uint64_t)tp | ((uint64_t)tm << 32) | ((uint64_t)(neg ? 1 : 0) << 63);
            v[d] = neg ? -t : t;
            crow[a] += 0.5 * ell;
            ccol[b] += 0.5 * ell;
        }
    }
    for (int a = 1; a < QM; ++a) {
        c[a - 1] = crow[a];
        c[(QM - 1) + a - 1] = ccol[a];
    }
}

// ---------------------------------------------------------------------------
// a2: x(0) = floor(u q) = floor((2U + 1) q / 2^25), U from phase INIT.
// ---------------------------------------------------------------------------
__global__ void k_init(int64_t n, int32_t C, const uint8_t *__restrict__ q,
                       uint8_t *__restrict__ x, uint32_t k0, uint32_t k1)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * C) return;
    const int64_t i = idx / C;
    const int c = (int)(idx - i * C);
    const Words w = philox4x32_10((uint32_t)i, (uint32_t)(i >> 32),
                                  (kPhaseInit << 30) | (uint32_t)(c >> 2), 0u, k0, k1);
    const uint32_t U = word_at(w, c & 3) >> 8;
    x[idx] = (uint8_t)(((2ull * U + 1ull) * q[i]) >> 25);
}

// Lane decomposition shared by the sweep kernels.
template <int LPI>
struct LaneMap {
    int lane;      // 0..63
    int64_t item;  // edge slot or node
    int c;         // chain
    int cb;        // chain block (LPI chains)
    __device__ __forceinline__ LaneMap(int32_t C)
    {
        constexpr int P = 64 / LPI;
        lane = threadIdx.x & 63;
        const int64_t wave =
            (int64_t)blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const int CB = (C + LPI - 1) / LPI;
        const int64_t group = wave / CB;
        cb = (int)(wave - group * CB);
        item = group * P + (P == 1 ? 0 : lane / LPI);
        c = cb * LPI + (LPI == 64 ? lane : lane % LPI);
    }
};

// ---------------------------------------------------------------------------
// a3: dual phase.  Every live edge, chain and entry d = (a-1)(q_dst-1)+(b-1):
// theta = [U >= T(k)], U from call sub = 16 c + d / 5, value d mod 5.
// The bits leave the wave as ballots, one 32-bit plane word per 32 chains.
// ---------------------------------------------------------------------------
template <int QM, int LPI>
__global__ __launch_bounds__(256) void k_dual(Graph g, uint32_t t)
{
    constexpr int D = dim_d(QM);
    constexpr int NCALL = (D + 4) / 5;
    const LaneMap<LPI> lm(g.C);
    const int64_t slot = lm.item;
    const bool in_range = slot < g.hwm;
    uint64_t uid = 0;
    if (in_range) uid = g.uid[slot];
    const bool live = uid != 0;
    const bool active = live && lm.c < g.C;
    uint64_t zbits = 0;
    if (active) {
        const int32_t s = g.src[slot], d = g.dst[slot];
        const uint32_t sq = g.sq[slot];
        const int qs = (int)(sq & 15u), qd = (int)(sq >> 4);
        const int xs = g.x[(int64_t)s * g.C + lm.c];
        const int xd = g.x[(int64_t)d * g.C + lm.c];
        const uint64_t *thr = reinterpret_cast<const uint64_t *>(g.params + slot * block_bytes(QM));
        const int De = (qs - 1) * (qd - 1);
        const uint32_t ulo = (uint32_t)uid, uhi = (uint32_t)(uid >> 32);
        int a = 1, b = 1;
#pragma unroll
        for (int k = 0; k < NCALL; ++k) {
            if (5 * k >= De) break;
            const Words w = philox4x32_10(ulo, uhi, (kPhaseDual << 30) | (uint32_t)(16 * lm.c + k), t,
                                          g.k0, g.k1);
            const uint32_t U[5] = {w.w0 >> 8, w.w1 >> 8, w.w2 >> 8, w.w3 >> 8, fifth_u24(w)};
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                const int dd = 5 * k + j;
                if (dd >= De) break;
                const uint64_t th = thr[dd];
                const uint32_t tp = (uint32_t)th & 0x1FFFFFFu;
                const uint32_t tm = (uint32_t)(th >> 32) & 0x1FFFFFFu;
                const bool neg = (th >> 63) != 0;
                const bool s1pos = (xs != a) != neg;
                const bool s2pos = (xd != b);
                const uint32_t T = (s1pos && s2pos) ? tp : ((!s1pos && !s2pos) ? tm : (1u << 23));
                if (U[j] >= T) zbits |= (1ull << dd);
                if (++b == qd) {
                    b = 1;
                    ++a;
                }
            }
        }
    }
    // Bit-planes out: item p owns ballot bits [p LPI, (p+1) LPI).
    const bool leader = live && ((LPI == 64) ? (lm.lane == 0) : (lm.lane % LPI == 0));
    uint32_t *zs = g.z + (uint64_t)(in_range ? slot : 0) * D * g.Wz;
#pragma unroll
    for (int dd = 0; dd < D; ++dd) {
        const uint64_t bal = __ballot((zbits >> dd) & 1ull);
        if (leader) {
            if (LPI == 64) {
                uint2 wv;
                wv.x = (uint32_t)bal;
                wv.y = (uint32_t)(bal >> 32);
                *reinterpret_cast<uint2 *>(zs + dd * g.Wz + 2 * lm.cb) = wv;
            } else {
                const int p0 = (lm.lane / LPI) * LPI;
                const uint64_t mask = (LPI >= 32) ? 0xFFFFFFFFull : ((1ull << (LPI & 31)) - 1ull);
                zs[dd * g.Wz] = (uint32_t)((bal >> p0) & mask);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// a4 + a5: primal phase and marginal counting.  Node i, chain c:
//   L(a) = lam(a) + sum over incident edges of the field of state a,
//   src side: c_row(a) + sum_b v_ab (1 - 2 theta_ab),
//   dst side: c_col(b) + sum_a t_ab (1 - 2 theta_ab), t = -|v|;
// then m = max L, w_a = e^(L(a) - m) (FP32 exp unless EXP64), F cumulative in
// FP64, x = min{a : u F_{q-1} < F_a}, u = (U + 0.5) 2^-24 from call
// (node, PRIMAL, c / 4, t), word c mod 4.
// ---------------------------------------------------------------------------
template <int QM, int LPI, bool EXP64>
__global__ __launch_bounds__(256) void k_primal(Graph g, uint32_t t, int count)
{
    constexpr int D = dim_d(QM);
    const LaneMap<LPI> lm(g.C);
    const int64_t node = lm.item;
    const bool valid = node < g.n;
    const bool active = valid && lm.c < g.C;
    int newx = -1;
    int qn = 0;
    if (valid) {
        qn = g.q[node];
        double L[QM];
#pragma unroll
        for (int a = 0; a < QM; ++a) L[a] = 0.0;
        const uint32_t off = g.inc_off[node], cnt = g.inc_cnt[node];
        const int w = lm.c >> 5;
        const uint32_t bit = (uint32_t)lm.c & 31u;
        for (uint32_t k = 0; k < cnt; ++k) {
            const uint32_t e = g.inc[off + k];
            if (e == kTomb) continue;
            const uint32_t slot = e >> 1;
            const uint32_t sq = g.sq[slot];
            const uint8_t *blk = g.params + (int64_t)slot * block_bytes(QM);
            const double *v = reinterpret_cast<const double *>(blk + 8 * D);
            const double *cc = reinterpret_cast<const double *>(blk + 16 * D);
            const uint32_t *zs = g.z + (uint64_t)slot * D * g.Wz + w;
            if ((e & 1u) == 0) {
                const int qo = (int)(sq >> 4);
#pragma unroll
                for (int a = 1; a < QM; ++a) {
                    if (a >= qn) break;
                    double s = cc[a - 1];
#pragma unroll
                    for (int b = 1; b < QM; ++b) {
                        if (b >= qo) break;
                        const int d = (a - 1) * (qo - 1) + (b - 1);
                        const uint32_t zb = (zs[d * g.Wz] >> bit) & 1u;
                        const double vv = v[d];
                        s += zb ? -vv : vv;
                    }
                    L[a] += s;
                }
            } else {
                const int qo = (int)(sq & 15u);
#pragma unroll
                for (int b = 1; b < QM; ++b) {
                    if (b >= qn) break;
                    double s = cc[(QM - 1) + b - 1];
#pragma unroll
                    for (int a = 1; a < QM; ++a) {
                        if (a >= qo) break;
                        const int d = (a - 1) * (qn - 1) + (b - 1);
                        const uint32_t zb = (zs[d * g.Wz] >> bit) & 1u;
                        const double tt = -fabs(v[d]);
                        s += zb ? -tt : tt;
                    }
                    L[b] += s;
                }
            }
        }
        const double *lam = g.lam + node * QM;
#pragma unroll
        for (int a = 0; a < QM; ++a)
            if (a < qn) L[a] += lam[a];
        double mx = L[0];
#pragma unroll
        for (int a = 1; a < QM; ++a)
            if (a < qn) mx = fmax(mx, L[a]);
        double F[QM];
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < QM; ++a) {
            if (a < qn) {
                double wgt;
                if (EXP64) {
                    wgt = exp(L[a] - mx);
                } else {
                    wgt = (double)exp2f((float)((L[a] - mx) * 1.4426950408889634074));
                }
                acc += wgt;
            }
            F[a] = acc;
        }
        const Words wd = philox4x32_10((uint32_t)node, (uint32_t)(node >> 32),
                                       (kPhasePrimal << 30) | (uint32_t)(lm.c >> 2), t, g.k0,
                                       g.k1);
        const uint32_t U = word_at(wd, lm.c & 3) >> 8;
        const double target = ((double)U + 0.5) * 5.9604644775390625e-08 * F[QM - 1];
        newx = qn - 1;
#pragma unroll
        for (int a = QM - 1; a >= 0; --a)
            if (a < qn && target < F[a]) newx = a;
        if (active) g.x[node * g.C + lm.c] = (uint8_t)newx;
    }
    if (count) {
        const bool leader = valid && ((LPI == 64) ? (lm.lane == 0) : (lm.lane % LPI == 0));
#pragma unroll
        for (int a = 0; a < QM; ++a) {
            const uint64_t bal = __ballot(active && newx == a);
            uint64_t mine = bal;
            if (LPI < 64) {
                const int p0 = (lm.lane / LPI) * LPI;
                mine = (bal >> p0) & ((LPI >= 64) ? ~0ull : ((1ull << (LPI & 63)) - 1ull));
            }
            if (leader && a < qn && mine != 0)
                atomicAdd(g.counts + node * QM + a, (uint32_t)__popcll(mine));
        }
    }
}

// ---------------------------------------------------------------------------
// Small kernels: edits, readout.
// ---------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// q (int32) -> uint8, log unaries -> FP64 [n][QM]; *bad = 1 if a used entry
// is not finite or q is out of range.
template <typename T>
__global__ void k_set_nodes(int64_t n, int32_t QM, const int32_t *__restrict__ q_in,
                            const T *__restrict__ lam_in, uint8_t *__restrict__ q,
                            double *__restrict__ lam, uint32_t *__restrict__ bad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int qi = q_in[i];
    if (qi < 2 || qi > QM) {
        atomicOr(bad, 2u);
        return;
    }
    q[i] = (uint8_t)qi;
    for (int a = 0; a < QM; ++a) {
        const double v = a < qi ? (double)lam_in[i * QM + a] : 0.0;
        if (!isfinite(v)) atomicOr(bad, 1u);
        lam[i * QM + a] = v;
    }
}

// New edges: slot arrays.
__global__ void k_slot_write(int64_t m, const int32_t *__restrict__ slots,
                             const int32_t *__restrict__ src_in, const int32_t *__restrict__ dst_in,
                             const uint64_t *__restrict__ uids, const uint8_t *__restrict__ q,
                             int32_t *__restrict__ src, int32_t *__restrict__ dst,
                             uint64_t *__restrict__ uid, uint8_t *__restrict__ sq,
                             int32_t *__restrict__ qs_out, int32_t *__restrict__ qd_out,
                             uint64_t *__restrict__ uid_out)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const int32_t s = slots[k], a = src_in[k], b = dst_in[k];
    src[s] = a;
    dst[s] = b;
    uid[s] = uids[k];
    const uint8_t qa = q[a], qb = q[b];
    sq[s] = (uint8_t)(qa | (qb << 4));
    qs_out[k] = qa;
    qd_out[k] = qb;
    if (uid_out) uid_out[k] = uids[k];
}

__global__ void k_slot_clear(int64_t m, const int32_t *__restrict__ slots, uint64_t *__restrict__ uid)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) uid[slots[k]] = 0;
}

// pool[idx[k]] = val[k]
__global__ void k_scatter_u32(int64_t m, const uint32_t *__restrict__ idx,
                              const uint32_t *__restrict__ val, uint32_t *__restrict__ pool)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) pool[idx[k]] = val[k];
}

// off[node[k]] = o[k], cnt[node[k]] = c[k]
__global__ void k_scatter_nodes(int64_t m, const uint32_t *__restrict__ node,
                                const uint32_t *__restrict__ o, const uint32_t *__restrict__ c,
                                uint32_t *__restrict__ off, uint32_t *__restrict__ cnt)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) {
        off[node[k]] = o[k];
        cnt[node[k]] = c[k];
    }
}

// theta of m edges (given by slot) for every chain: out [m][C], bit d.
__global__ void k_get_duals(int64_t m, int32_t C, int32_t D, int32_t Wz,
                            const int32_t *__restrict__ slots, const uint32_t *__restrict__ z,
                            uint64_t *__restrict__ out)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= m * C) return;
    const int64_t k = idx / C;
    const int c = (int)(idx - k * C);
    const uint32_t *zs = z + (uint64_t)slots[k] * D * Wz + (c >> 5);
    uint64_t bits = 0;
    for (int d = 0; d < D; ++d) bits |= (uint64_t)((zs[d * Wz] >> (c & 31)) & 1u) << d;
    out[idx] = bits;
}

// live uids in slot order: out[k] for the k-th live slot (prefix given by host)
__global__ void k_gather_u64(int64_t m, const int32_t *__restrict__ slots,
                             const uint64_t *__restrict__ v, uint64_t *__restrict__ out)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) out[k] = v[slots[k]];
}

__global__ void k_marginals(int64_t nq, const uint32_t *__restrict__ counts, double inv,
                            double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nq) out[i] = (double)counts[i] * inv;
}

}  // namespace pdg

// HIP kernels of the primal-dual Gibbs sweep for gfx950 (wave64).
//
// Work mapping.  Lanes are chains.  Items are edges in the dual phase and node
// quads (four consecutive nodes) in the primal phase.  With 33 or more chains
// (LPI = 64) an item owns whole waves (k_dual64: four edges per wave;
// k_primal64: one quad per wave), so everything per item -- endpoints,
// parameter block, incidence segment, mask words -- is wave-uniform and comes
// through scalar loads or LDS broadcasts, and a mask word is directly the
// lane mask of its chains.  With 17..32 chains the dual packs two edges per
// wave and k_primal32 splits one quad's records between the two half-waves;
// the generic k_dual / k_primal take 64 / LPI items per wave for fewer chains.
// Hubs (nodes with more than kHubThreshold incidences) are drawn by the hub
// kernels.
//
// Storage (device, all written by this library):
//   x       uint8  [n][C]                 node states, chain fastest
//   params  block  [slot]                 per-edge decomposition (layout below)
//   inc     uint32 pool                   per-node incidence segments
//                                         [off, off + cnt): slot << 1 | side
//                                         (side 0: node is src), or kTomb
//   rec_p   double [pool][D]              incidence records in the node's
//                                         orientation: entry (r-1)(QM-1) + (o-1)
//                                         for own state r, other end's state o
//                                         (h on the src side, |h| on the dst
//                                         side); zero for tombstones
//   base    double [n][QM]                lam plus the theta-free part c0 of
//                                         every incidence of the node, summed
//                                         in record order
//   rec_z   words  [pool][CB][D]          dual masks of each incidence record,
//                                         same entry order: with C <= 32 a
//                                         32-bit word per (record, entry), bit
//                                         c; with C > 32 a 64-bit word per
//                                         (record, block of 64 chains, entry).
//                                         With 17..32 chains and q_max >= 6
//                                         chain-major instead: [pool][C] 64-bit
//                                         words, bit 8 (r-1) + (o-1) of chain
//                                         c's word (zc_layout)
//   ipos    uint32 [slot][2]              record index of the src / dst side
//   counts  uint32 [n][QM]                marginal counters
// Parameter block of an edge (QM = q_max, D = (QM-1)^2, entry d = (a-1)(q_dst-1)+(b-1)):
//   sign  uint64          bit d set when the entry's log odds ratio is negative
//   thr   uint32 [D][2]   T+ * 256 - 1 and T- * 256 (thresholds on a 32-bit word
//                         whose top 24 bits are the draw's integer U)
//   h     double [D]      half the field increment of the src node's state a
//                         when theta = 1 (the dst node's state b gets 2|h|)
//   c0    double [2][QM-1] field of each state >= 1 when every dual of the
//                         edge is 0, src side then dst side
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "pdg_rng.hpp"

namespace pdg {

constexpr uint32_t kTomb = 0xFFFFFFFFu;

__host__ __device__ constexpr int dim_d(int qm) { return (qm - 1) * (qm - 1); }
__host__ __device__ constexpr int64_t off_thr(int) { return 8; }
__host__ __device__ constexpr int64_t off_h(int qm) { return 8 + 8 * (int64_t)dim_d(qm); }
__host__ __device__ constexpr int64_t off_c0(int qm) { return 8 + 16 * (int64_t)dim_d(qm); }
__host__ __device__ constexpr int64_t block_bytes(int qm)
{
    return 8 + 16 * (int64_t)dim_d(qm) + 16 * (int64_t)(qm - 1);
}
// The dual's part of a block: the sign word and the thresholds (its first
// off_h bytes).  A context keeps it per slot in an array of its own as well,
// so the dual kernels' lines carry no h or c0.
__host__ __device__ constexpr int64_t thr_bytes(int qm) { return off_h(qm); }

struct Graph {
    const uint8_t *__restrict__ q;        // [n] states per node
    const double *__restrict__ lam;       // [n][QM] log unaries (FP64)
    const double *__restrict__ base;      // [n][QM] lam + the c0 of the node's records
    const int32_t *__restrict__ src;      // [slots]
    const int32_t *__restrict__ dst;      // [slots]
    const uint64_t *__restrict__ uid;     // [slots], 0 = free slot
    const uint8_t *__restrict__ sq;       // [slots] q_src | q_dst << 4
    const uint8_t *__restrict__ params;   // [slots] parameter blocks
    const uint8_t *__restrict__ dparams;  // [slots] their sign words and thresholds (thr_bytes)
    const uint32_t *__restrict__ ipos;    // [slots][2] record index per side
    const uint32_t *__restrict__ inc_off; // [n]
    const uint32_t *__restrict__ inc_cnt; // [n]
    const uint32_t *__restrict__ inc;     // pool
    const double *__restrict__ rec_p;     // [pool][RP]
    uint32_t *__restrict__ rec_z;         // [pool][CB][D] words
    uint8_t *__restrict__ x;              // [n][C]
    uint32_t *__restrict__ counts;        // [n][QM]
    int64_t n;
    int64_t hwm;                          // slots [0, hwm) may be live
    int32_t C;
    int32_t CB;                           // blocks of 64 chains (1 when C <= 64)
    uint32_t heavy;                       // a node with more incidence entries is a hub,
                                          // drawn by the hub kernels (0: none)
    uint32_t k0, k1;                      // generator key
    RoundKeys rk;                         // its ten round keys
    const uint32_t *order;                // [n] node order of k_primal32z: its waves take the
                                          // nodes in this order, four at a time (null: id order)
    const uint32_t *tsrc;                 // replayed sweeps: the sweep counter in device
                                          // memory (null: the kernel argument t)
    int64_t burn;                         // counting starts after this sweep (with tsrc)
};

// Sweep counter of a phase kernel: the argument, or, in sweeps replayed from a
// captured HIP graph, the device counter the graph's tick kernel advances (and
// then whether this sweep is counted in the marginals).
__device__ __forceinline__ void sweep_args(const Graph &g, uint32_t &t, int &count)
{
    if (g.tsrc) {
        t = __builtin_amdgcn_readfirstlane(*g.tsrc);
        count = (int64_t)t > g.burn ? 1 : 0;
    }
}
__device__ __forceinline__ void sweep_args(const Graph &g, uint32_t &t)
{
    if (g.tsrc) t = __builtin_amdgcn_readfirstlane(*g.tsrc);
}

__host__ __device__ constexpr int rec_len(int qm) { return dim_d(qm); }
// Chain-major dual words: with 17..32 chains and records of 25 or more
// entries a record keeps one 64-bit word per chain (own state r in byte r-1,
// other state o in bit o-1 of it), so the primal reads a chain's duals of a
// whole record with one load and sums them through subset-sum tables
// (k_primal32z); otherwise one mask word per entry with a bit per chain.
__host__ __device__ constexpr bool zc_layout(int qm, int C) { return qm >= 6 && C >= 17 && C <= 32; }
// u32 words of dual masks per incidence record
__host__ __device__ inline int64_t rec_words(int qm, int C)
{
    if (zc_layout(qm, C)) return 2 * (int64_t)C;
    return C <= 32 ? (int64_t)dim_d(qm) : 2 * (int64_t)((C + 63) / 64) * dim_d(qm);
}
// Dual bit of chain c for padded entry dp (own state dp / (QM-1) + 1, other
// dp % (QM-1) + 1) of record r, in either layout.
__device__ __forceinline__ uint32_t rec_theta(const Graph &g, uint64_t r, int dp, int c, int qm)
{
    if (zc_layout(qm, g.C)) {
        const uint64_t w = reinterpret_cast<const uint64_t *>(g.rec_z)[r * (uint64_t)g.C + c];
        return (uint32_t)(w >> (8 * (dp / (qm - 1)) + dp % (qm - 1))) & 1u;
    }
    const int D = dim_d(qm);
    const uint64_t i = g.C <= 32 ? r * D + dp : ((r * g.CB + (c >> 6)) * D + dp) * 2 + ((c >> 5) & 1);
    return (g.rec_z[i] >> (c & 31)) & 1u;
}

// u32 index of the mask word holding chain c of padded entry dp of record r.
__device__ __forceinline__ uint64_t rec_zword(const Graph &g, uint64_t r, int dp, int c, int D)
{
    if (g.C <= 32) return r * D + dp;
    return ((r * g.CB + (c >> 6)) * D + dp) * 2 + ((c >> 5) & 1);
}

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
// p(theta = 0) = 1 / (1 + e^(t k)) takes three values and a draw compares the
// 24-bit integer U of its uniform u = (U + 0.5) 2^-24 with
// T = ceil(p0 2^24 - 0.5): theta = 0 iff U < T; T(0) = 2^23, T+ = T(2) >= 2^23,
// T- = T(-2) <= 2^23.
// Field of the one-hot bit of the src state a: 1/2 ell + sigma t (1 - 2 theta)
// = (1/2 ell + sigma t) + 2 theta h with h = -sigma t; of the dst state b:
// (1/2 ell + t) + 2 theta |h|.  The theta-free parts and the rescaling unaries
// L(a,0) - L(0,0), L(0,b) - L(0,0) are summed into c0.
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
// be null: identity).  *bad |= 1 if a used entry is not finite, |= 2 if a
// state count is outside [2, QM].
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
    uint32_t *thr = reinterpret_cast<uint32_t *>(blk + off_thr(QM));
    double *h = reinterpret_cast<double *>(blk + off_h(QM));
    double *c0 = reinterpret_cast<double *>(blk + off_c0(QM));
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
        thr[2 * d] = 0xFFFFFFFFu;
        thr[2 * d + 1] = 0u;
        h[d] = 0.0;
    }
    uint64_t sign = 0;
    for (int a = 1; a < qs; ++a) {
        for (int b = 1; b < qd; ++b) {
            const double ell = (double)L[a * QM + b] + L00 - (double)L[a * QM] - (double)L[b];
            const double t = log_tan_phi(ell);
            const bool neg = ell < 0.0;
            const uint32_t tp = threshold24(1.0 / (1.0 + exp(2.0 * t)));
            const uint32_t tm = threshold24(1.0 / (1.0 + exp(-2.0 * t)));
            const int d = (a - 1) * (qd - 1) + (b - 1);
            thr[2 * d] = (uint32_t)((uint64_t)tp * 256u - 1u);
            thr[2 * d + 1] = tm * 256u;
            const double st = neg ? -t : t;
            h[d] = -st;
            crow[a] += 0.5 * ell + st;
            ccol[b] += 0.5 * ell + t;
            if (neg) sign |= 1ull << d;
        }
    }
    *reinterpret_cast<uint64_t *>(blk) = sign;
    for (int a = 1; a < QM; ++a) {
        c0[a - 1] = crow[a];
        c0[(QM - 1) + a - 1] = ccol[a];
    }
}

// ---------------------------------------------------------------------------
// a2: x(0) = floor(u q) = floor((2U + 1) q / 2^25), U from phase INIT,
// call (node, c / 4), word c mod 4.
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
    int64_t item;  // edge slot or node quad of this lane
    int64_t base;  // item of lane 0 of the wave
    int c;         // chain
    int cb;        // chain block (LPI chains)
    __device__ __forceinline__ LaneMap(int32_t C)
        : LaneMap(C, (int64_t)blockIdx.x * (blockDim.x >> 6) +
                         __builtin_amdgcn_readfirstlane(threadIdx.x >> 6))
    {
    }
    // wave: index of this wave in the launch's item order
    __device__ __forceinline__ LaneMap(int32_t C, int64_t wave)
    {
        constexpr int P = 64 / LPI;
        lane = threadIdx.x & 63;
        const int CB = (C + LPI - 1) / LPI;
        const int64_t group = (CB == 1) ? wave : wave / CB;
        cb = (int)(wave - group * CB);
        base = group * P;
        item = base + (P == 1 ? 0 : lane / LPI);
        c = cb * LPI + (LPI == 64 ? lane : lane % LPI);
    }
};

// v_writelane_b32: set lane `lane` (uniform) of `old` to the uniform `value`.
extern "C" __device__ uint32_t pdg_writelane_i32(uint32_t value, uint32_t lane, uint32_t old)
    __asm("llvm.amdgcn.writelane.i32");

// 8 x 8 bit-matrix transpose of a 64-bit word (bit 8 r + c -> bit 8 c + r) by
// three delta swaps: a record word in the src orientation (byte = own state)
// becomes the same duals in the dst orientation.
__device__ __forceinline__ uint64_t transpose8x8(uint64_t x)
{
    uint64_t t = (x ^ (x >> 7)) & 0x00AA00AA00AA00AAull;
    x ^= t ^ (t << 7);
    t = (x ^ (x >> 14)) & 0x0000CCCC0000CCCCull;
    x ^= t ^ (t << 14);
    t = (x ^ (x >> 28)) & 0x00000000F0F0F0F0ull;
    x ^= t ^ (t << 28);
    return x;
}

// Wave-uniform lane mask -> per-lane predicate without VALU work.
__device__ __forceinline__ bool lane_bit(uint64_t mask)
{
    return __builtin_amdgcn_inverse_ballot_w64(mask);
}

// Marginal counters of a node quad whose wave owns them (one chain block):
// the 4 QM counters are contiguous (the array is padded to whole quads), so
// they are scalar-loaded (before any store of the kernel), raised by the
// popcounts of the state ballots, gathered into lanes j QM + a and written by
// one vector store.  `drawn` bit j: node j was drawn by this wave (qn[j] states);
// `chain` is this lane's chain predicate.
template <int QM>
__device__ __forceinline__ void count_quad(uint32_t *__restrict__ counts, int64_t quad,
                                           const int (&newx)[4], const int (&qn)[4],
                                           uint32_t drawn, bool chain, int lane)
{
    uint32_t *cq = counts + quad * 4 * QM;
    uint32_t row = 0;
    uint64_t wmask = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int a = 0; a < QM; ++a) {
            const uint32_t add =
                (uint32_t)__popcll(__ballot(((drawn >> j) & 1u) && chain && newx[j] == a));
            row = pdg_writelane_i32(cq[j * QM + a] + add, j * QM + a, row);
        }
        if ((drawn >> j) & 1u) wmask |= ((1ull << qn[j]) - 1ull) << (j * QM);
    }
    if (lane_bit(wmask)) cq[lane] = row;
}

// ---------------------------------------------------------------------------
// a3: dual phase.  Every live edge, chain and entry d = (a-1)(q_dst-1)+(b-1):
// theta = [U >= T(k)], U from call (uid, DUAL, 16 c + d / 5, t), value d mod 5.
// The five values of a call are kept in "W form" (U in the top 24 bits of a
// 32-bit word), so the three candidate thresholds are single compares:
// U >= T+  <=>  W > T+ 256 - 1,  U >= 2^23  <=>  W >= 2^31,  U >= T-  <=>  W >= T- 256.
// The compare results are lane masks; the (y, y', sigma) case analysis is mask
// logic, and the ballot of theta is the dual bit-plane word.
// UQ: every node has q_max states (compile-time entry loops).
// ---------------------------------------------------------------------------
// STG: the caller is a launch of 256-thread blocks (four waves), so each wave
// may stage its items' dual parameters in an LDS region of its own.
template <int QM, int LPI, bool UQ, bool STG = false>
__device__ __forceinline__ void dual_wave(const Graph &g, uint32_t t, const LaneMap<LPI> lm)
{
    static_assert(LPI <= 32, "33 or more chains: k_dual64");
    constexpr int D = dim_d(QM);
    constexpr int NCALL = (D + 4) / 5;
    constexpr int P = 64 / LPI;                      // items (edge slots) per wave
    // LPI >= 8 and records of 4 or more words: the mask words of the wave's P
    // items are gathered into lanes p D + d and stored record by record (one
    // contiguous run per record); otherwise the first lane of each item
    // stores its words, with the record addresses loaded before the draws
    // ZC (17..32 chains, q_max >= 6): each lane keeps its chain's words of
    // both records (chain-major layout) and stores them at the end
    constexpr bool ZC = LPI == 32 && QM >= 6;
    constexpr bool GATHER = !ZC && (LPI >= 32 || (LPI >= 8 && D >= 4));
    constexpr int NW = GATHER ? P * D : 1;
    constexpr int NREG = (NW + 63) / 64;
    constexpr uint32_t WMASK = LPI >= 32 ? 0xFFFFFFFFu : (1u << LPI) - 1u;
    const int64_t slot = lm.item;
    const bool in_range = slot < g.hwm;
    const int64_t sl = in_range ? slot : 0;
    const uint64_t uid = in_range ? g.uid[sl] : 0ull;
    const bool live = uid != 0;
    const bool active = live && lm.c < g.C;
    int qs = QM, qd = QM;
    if (!UQ && live) {
        const uint32_t sq = g.sq[sl];
        qs = (int)(sq & 15u);
        qd = (int)(sq >> 4);
    }
    int xs = -1, xd = -1;
    if (active) {
        xs = g.x[(int64_t)g.src[sl] * g.C + lm.c];
        xd = g.x[(int64_t)g.dst[sl] * g.C + lm.c];
    }
    const uint8_t *blk = g.dparams + sl * thr_bytes(QM);
    const uint64_t sign = *reinterpret_cast<const uint64_t *>(blk);
    const uint32_t *thr = reinterpret_cast<const uint32_t *>(blk + off_thr(QM));
    // With 8 to 32 chains per item the dual parameters of the wave's P items
    // (P (8 + 8 D) bytes; the slots are consecutive) are staged in the wave's
    // LDS region by 16-byte loads, one or a few per lane, so the per-entry
    // thresholds are LDS broadcasts instead of a chain of global loads.  The
    // block array is padded to whole groups of 8 slots, so every item's row
    // is in bounds.
    constexpr int TW = (int)(thr_bytes(QM) / 4);  // dwords per slot
    constexpr bool STAGE = STG && LPI >= 8;
    constexpr int NCH = P * (1 + D) / 2;           // 16-byte chunks of the P rows
    __shared__ __align__(16) uint32_t sthr[4][STAGE ? P * TW : 4];
    const uint32_t *lthr = thr;
    if constexpr (STAGE) {
        uint32_t *my = sthr[__builtin_amdgcn_readfirstlane(threadIdx.x >> 6) & 3];
        const uint4 *src = reinterpret_cast<const uint4 *>(g.dparams + lm.base * thr_bytes(QM));
#pragma unroll
        for (int i = 0; i < (NCH + 63) / 64; ++i) {
            const int k = i * 64 + lm.lane;
            if (k < NCH) reinterpret_cast<uint4 *>(my)[k] = src[k];
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        lthr = my + (lm.lane / LPI) * TW + 2;
    }
    const int De = UQ ? D : (qs - 1) * (qd - 1);
    const uint32_t ulo = (uint32_t)uid, uhi = (uint32_t)(uid >> 32);
    const uint64_t mact = __ballot(active);
    // with two items per wave their sign words are taken to scalar registers,
    // so the per-entry sign mask is scalar work
    uint32_t sg[2][2] = {{0u, 0u}, {0u, 0u}};  // [item][word]
    if constexpr (LPI == 32) {
        const uint32_t slo = (uint32_t)sign, shi = (uint32_t)(sign >> 32);
        sg[0][0] = __builtin_amdgcn_readlane(slo, 0);
        sg[0][1] = __builtin_amdgcn_readlane(shi, 0);
        sg[1][0] = __builtin_amdgcn_readlane(slo, 32);
        sg[1][1] = __builtin_amdgcn_readlane(shi, 32);
    }
    // lane masks of the one-hot bits y = [x_src = a], y' = [x_dst = b]
    uint64_t mya[QM], myb[QM];
#pragma unroll
    for (int v = 1; v < QM; ++v) {
        mya[v] = UQ ? __ballot(xs == v) : 0ull;
        myb[v] = UQ ? __ballot(xd == v) : 0ull;
    }
    uint32_t outr[NREG];
#pragma unroll
    for (int r = 0; r < NREG; ++r) outr[r] = 0u;
    uint32_t zs[2] = {0u, 0u};  // ZC: this chain's src record word
    const bool leader = !ZC && live && (lm.lane % LPI == 0);
    // records of the two endpoints receive the masks
    const uint64_t r0 = live ? g.ipos[2 * sl] : 0ull, r1 = live ? g.ipos[2 * sl + 1] : 0ull;
    int a = 1, b = 1;
#pragma unroll
    for (int k = 0; k < NCALL; ++k) {
        if (!UQ && __ballot(5 * k < De) == 0) break;
        const Words w = philox4x32_10(ulo, uhi, (kPhaseDual << 30) | (uint32_t)(16 * lm.c + k), t,
                                      g.rk);
        const uint32_t W[5] = {w.w0, w.w1, w.w2, w.w3,
                               fifth_w(w)};
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            const int dd = 5 * k + j;
            if (dd >= D) break;
            // k = sigma (1 - 2y) + (1 - 2y') is +2 where yh = y ^ [sigma < 0] and y'
            // are both 0, -2 where both are 1, else 0.  The compare masks nest
            // (U >= T+ implies U >= 2^23 implies U >= T-), so
            // theta = cp | (ch & (yh | y')) | (cm & yh & y').
            // Lanes of absent chains produce bits that nothing reads.
            const uint64_t ya = UQ ? mya[dd / (QM - 1) + 1] : __ballot(xs == a);
            const uint64_t yb = UQ ? myb[dd % (QM - 1) + 1] : __ballot(xd == b);
            uint64_t neg;
            if constexpr (LPI == 32) {
                const uint32_t n0 = 0u - ((sg[0][dd >> 5] >> (dd & 31)) & 1u);
                const uint32_t n1 = 0u - ((sg[1][dd >> 5] >> (dd & 31)) & 1u);
                neg = ((uint64_t)n1 << 32) | n0;
            } else {
                neg = __ballot(((sign >> dd) & 1ull) != 0);
            }
            const uint64_t yh = ya ^ neg;
            const uint32_t tp8m1 = lthr[2 * dd], tm8 = lthr[2 * dd + 1];
            const uint64_t cp = __ballot(W[j] > tp8m1);          // U >= T+
            const uint64_t cm = __ballot(W[j] >= tm8);           // U >= T-
            const uint64_t ch = __ballot(W[j] >= 0x80000000u);   // U >= 2^23
            uint64_t zm = cp | (ch & (yh | yb)) | (cm & yh & yb);
            if (!UQ) zm &= __ballot(dd < De) & mact;
            if constexpr (ZC) {
                // bit 8 (a-1) + (b-1) of the src word (the dst word is its
                // transpose, formed at the end)
                const int ai = UQ ? dd / (QM - 1) : a - 1, bi = UQ ? dd % (QM - 1) : b - 1;
                const uint32_t th = lane_bit(zm) ? 1u : 0u;
                const int ps = 8 * ai + bi;
                if (UQ) {
                    zs[ps >> 5] |= th << (ps & 31);
                } else {
                    // entries past the edge's own carry th = 0
                    const uint32_t vs = th << (ps & 31);
                    zs[0] |= ps < 32 ? vs : 0u;
                    zs[1] |= ps < 32 ? 0u : vs;
                }
            } else if (GATHER) {
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    const int idx = p * D + dd;
                    outr[idx >> 6] = pdg_writelane_i32((uint32_t)(zm >> (p * LPI)) & WMASK,
                                                       idx & 63, outr[idx >> 6]);
                }
            } else if (leader && (UQ || dd < De)) {
                const int p0 = (lm.lane / LPI) * LPI;
                const uint32_t wv = (uint32_t)((zm >> p0) & ((1ull << (LPI & 31)) - 1ull));
                const int ai = UQ ? dd / (QM - 1) : a - 1, bi = UQ ? dd % (QM - 1) : b - 1;
                g.rec_z[r0 * D + ai * (QM - 1) + bi] = wv;
                g.rec_z[r1 * D + bi * (QM - 1) + ai] = wv;
            }
            if (!UQ) {
                if (++b == qd) {
                    b = 1;
                    ++a;
                }
            }
        }
        // ZC: fold each call's bits into the words here (left alone, the
        // compiler defers every select to the end, and the compare masks of
        // all entries, held until then, exceed the scalar registers)
        if constexpr (ZC) {
            // (an identity DPP move: opaque to the compiler, costs one VALU)
            zs[0] = __builtin_amdgcn_mov_dpp((int)zs[0], 0xE4, 0xF, 0xF, false);
            zs[1] = __builtin_amdgcn_mov_dpp((int)zs[1], 0xE4, 0xF, 0xF, false);
        }
    }
    // GATHER: the gathered mask words go out to both records, each in its
    // node's orientation: (a-1)(QM-1) + (b-1) in the src record, (b-1)(QM-1) +
    // (a-1) in the dst record; lane p D + d of register r (index 64 r + lane)
    // holds item p's word of entry d, so consecutive lanes fill one record.
    if constexpr (ZC) {
        if (active) {
            const uint64_t ws = ((uint64_t)zs[1] << 32) | zs[0];
            uint64_t *z = reinterpret_cast<uint64_t *>(g.rec_z);
            z[r0 * (uint64_t)g.C + lm.c] = ws;
            z[r1 * (uint64_t)g.C + lm.c] = transpose8x8(ws);
        }
        return;
    }
    auto padded = [&](int dd, int qdv) -> int {
        return (dd / (qdv - 1)) * (QM - 1) + dd % (qdv - 1);
    };
    auto transposed = [&](int dd, int qdv) -> int {
        return (dd % (qdv - 1)) * (QM - 1) + dd / (qdv - 1);
    };
    if (GATHER) {
#pragma unroll
        for (int r = 0; r < NREG; ++r) {
            const int idx = 64 * r + lm.lane;
            if (idx < NW) {
                const int p = idx / D, dd = idx - p * D;
                const int64_t sp = lm.base + p;
                if (sp < g.hwm && g.uid[sp] != 0) {
                    int qdp = QM, Dep = D;
                    if (!UQ) {
                        const uint32_t sqp = g.sq[sp];
                        qdp = (int)(sqp >> 4);
                        Dep = ((int)(sqp & 15u) - 1) * (qdp - 1);
                    }
                    if (UQ || dd < Dep) {
                        const int dp = UQ ? dd : padded(dd, qdp);
                        const int dt = transposed(dd, UQ ? QM : qdp);
                        g.rec_z[(uint64_t)g.ipos[2 * sp] * D + dp] = outr[r];
                        g.rec_z[(uint64_t)g.ipos[2 * sp + 1] * D + dt] = outr[r];
                    }
                }
            }
        }
    }
}

template <int QM, int LPI, bool UQ>
__global__ __launch_bounds__(256) void k_dual(Graph g, uint32_t t)
{
    sweep_args(g, t);
    dual_wave<QM, LPI, UQ, true>(g, t, LaneMap<LPI>(g.C));
}

// ---------------------------------------------------------------------------
// a3 for binary records (q_max 2) with 8 or 16 chains: one draw per edge and
// chain, so a wave of dual_wave is a chain of dependent loads (slot, endpoints,
// their states) around a single generator call.  Here a wave takes E item
// groups (E P consecutive slots) and issues the loads of all of them before
// drawing, so E such chains are in flight per wave.  Draws, mask logic and
// stores are dual_wave's (entry d = 0, value 0 of call (uid, DUAL, 16 c, t)).
// ---------------------------------------------------------------------------
constexpr int kBinaryGroupsPerWave = 4;

template <int LPI, bool UQ, int E>
__global__ __launch_bounds__(256) void k_dual_bin(Graph g, uint32_t t)
{
    static_assert(LPI == 8 || LPI == 16, "binary dual: 8 or 16 chains per item");
    sweep_args(g, t);
    constexpr int P = 64 / LPI;
    constexpr uint32_t WMASK = (1u << LPI) - 1u;
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) +
                         __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c = lane % LPI;
    const int pl = lane / LPI;
    uint64_t uid[E];
    int32_t es[E], ed[E];
    uint32_t tp[E], tm[E], r0[E], r1[E];
    bool neg[E];
    int De[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int64_t sl = (wave * E + e) * P + pl;
        const bool in_range = sl < g.hwm;
        uid[e] = in_range ? g.uid[sl] : 0ull;
        const bool live = uid[e] != 0;
        es[e] = 0;
        ed[e] = 0;
        tp[e] = 0;
        tm[e] = 0;
        r0[e] = 0;
        r1[e] = 0;
        neg[e] = false;
        De[e] = 1;
        if (live) {
            es[e] = g.src[sl];
            ed[e] = g.dst[sl];
            const uint8_t *blk = g.dparams + sl * thr_bytes(2);
            neg[e] = (*reinterpret_cast<const uint64_t *>(blk) & 1ull) != 0;
            const uint32_t *thr = reinterpret_cast<const uint32_t *>(blk + off_thr(2));
            tp[e] = thr[0];
            tm[e] = thr[1];
            r0[e] = g.ipos[2 * sl];
            r1[e] = g.ipos[2 * sl + 1];
            if (!UQ) {
                const uint32_t sq = g.sq[sl];
                De[e] = ((int)(sq & 15u) - 1) * ((int)(sq >> 4) - 1);
            }
        }
    }
    int xs[E], xd[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        xs[e] = -1;
        xd[e] = -1;
        if (uid[e] != 0 && c < g.C) {
            xs[e] = g.x[(int64_t)es[e] * g.C + c];
            xd[e] = g.x[(int64_t)ed[e] * g.C + c];
        }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const bool live = uid[e] != 0;
        const bool active = live && c < g.C;
        const Words w = philox4x32_10((uint32_t)uid[e], (uint32_t)(uid[e] >> 32),
                                      (kPhaseDual << 30) | (uint32_t)(16 * c), t, g.rk);
        const uint64_t ya = __ballot(xs[e] == 1), yb = __ballot(xd[e] == 1);
        const uint64_t yh = ya ^ __ballot(neg[e]);
        const uint64_t cp = __ballot(w.w0 > tp[e]);          // U >= T+
        const uint64_t cm = __ballot(w.w0 >= tm[e]);         // U >= T-
        const uint64_t ch = __ballot(w.w0 >= 0x80000000u);   // U >= 2^23
        uint64_t zm = cp | (ch & (yh | yb)) | (cm & yh & yb);
        if (!UQ) zm &= __ballot(0 < De[e]) & __ballot(active);
        if (live && c == 0 && (UQ || De[e] > 0)) {
            const uint32_t wv = (uint32_t)(zm >> (pl * LPI)) & WMASK;
            g.rec_z[r0[e]] = wv;
            g.rec_z[r1[e]] = wv;
        }
    }
}

// ---------------------------------------------------------------------------
// a3 with 33 or more chains: a wave takes E consecutive edge slots for one
// block of 64 chains.  The slot metadata of all E edges comes in one batch of
// scalar loads and their endpoint states in one batch of gathers; the
// parameter block of the next edge is requested while the current edge is
// drawn, and the mask words of all E edges are stored at the end, so every
// load precedes every store.  Draws and mask logic are those of k_dual.
// The slot arrays are padded to a multiple of E; free slots have uid 0.
// ---------------------------------------------------------------------------
constexpr int kDualEdgesPerWave = 4;      // default; the tuner picks 2, 4 or 8
constexpr int kMaxDualEdgesPerWave = 8;   // slot arrays are padded to a multiple of this

template <int QM>
struct DualParams {
    uint64_t sign;
    uint32_t thr[2 * dim_d(QM)];
};

template <int QM, bool UQ, int E>
__global__ __launch_bounds__(256) void k_dual64(Graph g, uint32_t t)
{
    sweep_args(g, t);
    constexpr int D = dim_d(QM);
    constexpr int NCALL = (D + 4) / 5;
    constexpr int NW = 2 * D;  // mask half-words of one edge
    constexpr int NREG = (NW + 63) / 64;
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) +
                         __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t group = (g.CB == 1) ? wave : wave / g.CB;
    const int cb = (int)(wave - group * g.CB);
    const int c = cb * 64 + lane;
    const bool cvalid = c < g.C;
    const int64_t s0 = group * E;
    if (s0 >= g.hwm) return;
    uint64_t uid[E];
    int32_t sv[E], dv[E];
    uint32_t r0[E], r1[E], sq[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        uid[e] = g.uid[s0 + e];
        sv[e] = g.src[s0 + e];
        dv[e] = g.dst[s0 + e];
        r0[e] = g.ipos[2 * (s0 + e)];
        r1[e] = g.ipos[2 * (s0 + e) + 1];
        sq[e] = UQ ? 0u : (uint32_t)g.sq[s0 + e];
    }
    // endpoint states, loaded unconditionally (free slots hold valid stale
    // endpoints, or 0; lanes past C read chain 0 and their bits are masked)
    const int cx = cvalid ? c : 0;
    int xs[E], xd[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        xs[e] = g.x[(int64_t)sv[e] * g.C + cx];
        xd[e] = g.x[(int64_t)dv[e] * g.C + cx];
    }
    const uint64_t mact = __ballot(cvalid);
    auto load_params = [&](int64_t slot, DualParams<QM> &p) {
        const uint8_t *blk = g.dparams + slot * thr_bytes(QM);
        p.sign = *reinterpret_cast<const uint64_t *>(blk);
        const uint32_t *thr = reinterpret_cast<const uint32_t *>(blk + off_thr(QM));
#pragma unroll
        for (int i = 0; i < 2 * D; ++i) p.thr[i] = thr[i];
    };
    // touch the E edges' sign words and thresholds (contiguous) with vector
    // loads, all lines in flight at once, so the scalar loads of the edge loop
    // hit L2
    uint32_t sink;
    {
        constexpr int64_t BB = thr_bytes(QM);
        const uint64_t pb = (uint64_t)s0 * BB, pe = pb + (uint64_t)E * BB;
        const uint64_t pa = (pb & ~(uint64_t)127) + 128 * (uint64_t)lane;
        sink = pa < pe ? *reinterpret_cast<const uint32_t *>(g.dparams + pa) : 0u;
    }
    // and the record indices, which the stores at the end read
    const uint32_t sink_ip = lane == 63 ? g.ipos[2 * s0] : 0u;
    uint32_t outr[E][NREG];
#pragma unroll
    for (int e = 0; e < E; ++e) {
#pragma unroll
        for (int r = 0; r < NREG; ++r) outr[e][r] = 0u;
        if (uid[e] != 0) {
            DualParams<QM> cur;
            load_params(s0 + e, cur);
            int qs = QM, qd = QM;
            if (!UQ) {
                qs = (int)(sq[e] & 15u);
                qd = (int)(sq[e] >> 4);
            }
            const int De = UQ ? D : (qs - 1) * (qd - 1);
            const uint32_t ulo = (uint32_t)uid[e], uhi = (uint32_t)(uid[e] >> 32);
            uint64_t mya[QM], myb[QM];
#pragma unroll
            for (int v = 1; v < QM; ++v) {
                mya[v] = __ballot(xs[e] == v);
                myb[v] = __ballot(xd[e] == v);
            }
            int an = 1, bn = 1;  // entry (a, b) of the next draw when not UQ
#pragma unroll
            for (int k = 0; k < NCALL; ++k) {
                if (!UQ && 5 * k >= De) break;
                const Words w = philox4x32_10(ulo, uhi, (kPhaseDual << 30) | (uint32_t)(16 * c + k),
                                              t, g.rk);
                const uint32_t W[5] = {w.w0, w.w1, w.w2, w.w3,
                                       fifth_w(w)};
#pragma unroll
                for (int j = 0; j < 5; ++j) {
                    const int dd = 5 * k + j;
                    if (dd >= D) break;
                    int ai = an, bi = bn;  // 1-based entry (a, b) of draw dd
                    if (UQ) {
                        ai = dd / (QM - 1) + 1;
                        bi = dd % (QM - 1) + 1;
                    } else if (++bn == qd) {
                        bn = 1;
                        ++an;
                    }
                    uint64_t ya = 0, yb = 0;
#pragma unroll
                    for (int v = 1; v < QM; ++v) {
                        if (v == ai) ya = mya[v];
                        if (v == bi) yb = myb[v];
                    }
                    const uint64_t neg = 0ull - ((cur.sign >> dd) & 1ull);
                    const uint64_t yh = ya ^ neg;
                    const uint64_t cp = __ballot(W[j] > cur.thr[2 * dd]);        // U >= T+
                    const uint64_t cm = __ballot(W[j] >= cur.thr[2 * dd + 1]);   // U >= T-
                    const uint64_t ch = __ballot(W[j] >= 0x80000000u);          // U >= 2^23
                    uint64_t zm = cp | (ch & (yh | yb)) | (cm & yh & yb);
                    zm &= mact;
                    if (!UQ && dd >= De) zm = 0;
                    outr[e][(2 * dd) >> 6] =
                        pdg_writelane_i32((uint32_t)zm, (2 * dd) & 63, outr[e][(2 * dd) >> 6]);
                    outr[e][(2 * dd + 1) >> 6] = pdg_writelane_i32(
                        (uint32_t)(zm >> 32), (2 * dd + 1) & 63, outr[e][(2 * dd + 1) >> 6]);
                }
            }
        }
    }
    asm volatile("" ::"v"(sink), "v"(sink_ip));
    // lane 2d + h holds half h of entry d's mask; the src record takes entry
    // (a-1)(QM-1) + (b-1), the dst record (b-1)(QM-1) + (a-1)
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int qd = UQ ? QM : (int)(sq[e] >> 4);
        const int De = UQ ? D : ((int)(sq[e] & 15u) - 1) * (qd - 1);
        uint32_t *z0 = g.rec_z + ((uint64_t)r0[e] * g.CB + cb) * 2 * D;
        uint32_t *z1 = g.rec_z + ((uint64_t)r1[e] * g.CB + cb) * 2 * D;
#pragma unroll
        for (int r = 0; r < NREG; ++r) {
            const int idx = 64 * r + lane;
            const int dd = idx >> 1;
            if (uid[e] != 0 && idx < NW && dd < De) {
                const int ai = dd / (qd - 1), bi = dd % (qd - 1);
                z0[2 * (ai * (QM - 1) + bi) + (idx & 1)] = outr[e][r];
                z1[2 * (bi * (QM - 1) + ai) + (idx & 1)] = outr[e][r];
            }
        }
    }
}

// Categorical draw of one node from its field L (FP64): m = max L, weights
// e^(L(a) - m) (FP32 exp unless EXP64: the hardware's 2^x on (L(a) - m) log2 e,
// whose relative error is about 1e-7; weights below 2^-126 may flush to 0), F
// cumulative in FP64, x = min{a : u F_{q-1} < F_a} with u = (U + 0.5) 2^-24.
template <int QM, bool UQ, bool EXP64>
__device__ __forceinline__ int draw_node(const double (&L)[QM], int qn, uint32_t U)
{
    double mx = L[0];
#pragma unroll
    for (int a = 1; a < QM; ++a)
        if (UQ || a < qn) mx = fmax(mx, L[a]);
    double F[QM];
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < QM; ++a) {
        if (UQ || a < qn) {
            double wgt;
            if (EXP64)
                wgt = exp(L[a] - mx);
            else
                wgt = (double)__builtin_amdgcn_exp2f((float)((L[a] - mx) * 1.4426950408889634074));
            acc += wgt;
        }
        F[a] = acc;
    }
    const double target = ((double)U + 0.5) * 5.9604644775390625e-08 * F[QM - 1];
    int xn = qn - 1;
#pragma unroll
    for (int a = QM - 1; a >= 0; --a)
        if ((UQ || a < qn) && target < F[a]) xn = a;
    return xn;
}

// ---------------------------------------------------------------------------
// a4 + a5 with 33 or more chains: a wave takes one node quad for one block of
// 64 chains.  The h values of the quad's records are staged into the wave's
// LDS region with one batch of 16-byte vector loads (all four nodes in flight
// together) and read back as broadcasts; the dual masks, which are lane masks
// used directly as FMA selects, come through scalar loads, two records per
// wait, after their lines were touched into L2.  A node with more records
// than a staged chunk holds is walked chunk by chunk.
// ---------------------------------------------------------------------------
// eight waves per SIMD where the register budget of eight waves costs no
// spills (q_max <= 5): the kernel waits on memory
template <int QM, bool UQ, bool EXP64>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(QM <= 5 ? 8 : 1))) void k_primal64(
    Graph g, uint32_t t, int count)
{
    sweep_args(g, t, count);
    constexpr int D = dim_d(QM);
    constexpr int RP = rec_len(QM);                         // doubles per record
    constexpr int NLD = D <= 16 ? 1 : 2;                    // 16-byte loads per lane and node
    constexpr int CHB = 1024 * NLD;                         // staged bytes per node
    constexpr int K = (CHB - 16) / (8 * RP);                // records per chunk
    static_assert(K >= 1, "chunk holds no record");
    __shared__ __align__(16) uint8_t stage[4][4][CHB];      // [wave of block][node][bytes]
    const LaneMap<64> lm(g.C);
    const int lane = lm.lane;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t quad = lm.item;
    const bool cvalid = lm.c < g.C;
    uint32_t off[4] = {0, 0, 0, 0}, cnt[4] = {0, 0, 0, 0};
    uint32_t hub = 0;  // bit j: node j is a hub (drawn by the hub kernels)
    if (quad * 4 < g.n) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            off[j] = g.inc_off[quad * 4 + j];
            cnt[j] = g.inc_cnt[quad * 4 + j];
            if (g.heavy && cnt[j] > g.heavy) {
                hub |= 1u << j;
                cnt[j] = 0;
            }
        }
    }
    // records [first, first + nrec) of node j into its LDS region; returns the
    // byte shift of the first record (the copy starts 16-byte aligned; the
    // record array is padded past its end)
    auto stage_chunk = [&](int j, uint32_t first, uint32_t nrec) -> uint32_t {
        const uint64_t start = ((uint64_t)off[j] + first) * (RP * 8);
        const uint64_t a16 = start & ~(uint64_t)15;
        const uint32_t shift = (uint32_t)(start - a16);
        const uint32_t bytes = shift + nrec * (RP * 8);
        const uint8_t *src = reinterpret_cast<const uint8_t *>(g.rec_p) + a16;
#pragma unroll
        for (int i = 0; i < NLD; ++i) {
            const uint32_t o = (uint32_t)(i * 64 + lane) * 16;
            if (o < bytes)
                *reinterpret_cast<uint4 *>(&stage[wib][j][o]) =
                    *reinterpret_cast<const uint4 *>(src + o);
        }
        return shift;
    };
    const int64_t zstride = (int64_t)g.CB * D * 2;  // u32 per record
    uint32_t sink_z, sink_b;  // touch loads, issued with the staging loads
    // the first chunk of all four nodes: every lane loads its pieces of the
    // four regions before any is written (lanes past a chunk's end re-read its
    // first piece, in bounds as the record array is padded), so the four
    // loads share one wait instead of one each.  Only when one of the nodes
    // has a record: a context without edges has no record arrays at all.
    uint32_t shift[4] = {0u, 0u, 0u, 0u};
    sink_z = sink_b = 0u;
    if ((cnt[0] | cnt[1] | cnt[2] | cnt[3]) != 0u) {
        uint4 v[4][NLD];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t nrec = cnt[j] < K ? cnt[j] : K;
            const uint64_t start = (uint64_t)off[j] * (RP * 8);
            const uint64_t a16 = start & ~(uint64_t)15;
            shift[j] = (uint32_t)(start - a16);
            const uint32_t bytes = shift[j] + nrec * (RP * 8);
            const uint8_t *src = reinterpret_cast<const uint8_t *>(g.rec_p) + a16;
#pragma unroll
            for (int i = 0; i < NLD; ++i) {
                const uint32_t o = (uint32_t)(i * 64 + lane) * 16;
                v[j][i] = *reinterpret_cast<const uint4 *>(src + (o < bytes ? o : 0u));
            }
        }
        // mask lines of the four segments into L2 (lane (j, l): line l of node
        // j; lanes past a segment's end touch its first line again)
        {
            const int j = lane >> 4, l = lane & 15;
            const uint32_t oj = j == 0 ? off[0] : j == 1 ? off[1] : j == 2 ? off[2] : off[3];
            const uint32_t cj = j == 0 ? cnt[0] : j == 1 ? cnt[1] : j == 2 ? cnt[2] : cnt[3];
            const uint64_t zb = (uint64_t)oj * zstride * 4, ze = zb + (uint64_t)cj * zstride * 4;
            const uint64_t z0 = zb & ~(uint64_t)127, za = z0 + 128 * (uint64_t)l;
            sink_z = *reinterpret_cast<const uint32_t *>(reinterpret_cast<const uint8_t *>(g.rec_z) +
                                                         (za < ze ? za : z0));
        }
        // and the quad's base and counter rows (read later through scalar loads;
        // lanes 0..31: lines of the 32 QM base bytes, lanes 32..63: of the 16 QM
        // counter bytes, or the base again when nothing is counted)
        {
            const int64_t qc = quad * 4 < g.n ? quad : 0;
            const bool cpart = lane >= 32 && count;
            const uint64_t b0 = cpart ? (uint64_t)(g.counts + qc * 4 * QM) : (uint64_t)(g.base + qc * 4 * QM);
            const uint64_t b1 = b0 + (cpart ? 16 * QM : 32 * QM);
            const uint64_t l0 = b0 & ~(uint64_t)127, ba = l0 + 128 * (uint64_t)(lane & 31);
            sink_b = *reinterpret_cast<const uint32_t *>(ba < b1 ? ba : l0);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int i = 0; i < NLD; ++i)
                *reinterpret_cast<uint4 *>(&stage[wib][j][(i * 64 + lane) * 16]) = v[j][i];
    }
    const Words wq = philox4x32_10((uint32_t)quad, (uint32_t)(quad >> 32),
                                   (kPhasePrimal << 30) | (uint32_t)lm.c, t, g.rk);
    const uint32_t Wn[4] = {wq.w0, wq.w1, wq.w2, wq.w3};
    int newx[4], qnv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t node = quad * 4 + j;
        newx[j] = -1;
        qnv[j] = 0;
        if (node >= g.n || ((hub >> j) & 1u)) continue;
        const int qn = UQ ? QM : (int)g.q[node];
        qnv[j] = qn;
        // the theta-free part (lam and every c0) is the node's base, read by
        // vector loads from an opaque copy of the node id (an identity DPP
        // move), so that its latency overlaps the first mask loads' wait
        // instead of adding a scalar wait of its own
        const int64_t nv = (int64_t)(uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)node, 0xE4, 0xF, 0xF, false);
        double L[QM];
#pragma unroll
        for (int a = 0; a < QM; ++a) L[a] = (UQ || a < qn) ? g.base[nv * QM + a] : 0.0;
        auto record = [&](const double *h, const uint64_t *z) {
#pragma unroll
            for (int s = 1; s < QM; ++s) {
                if (!UQ && s >= qn) break;
                double acc = L[s];
#pragma unroll
                for (int o = 1; o < QM; ++o) {
                    // acc + 2 theta h in one FMA: the factor is 0.0 or 2.0 (a
                    // select of inline constants) and 2 h is exact
                    const int dp = (s - 1) * (QM - 1) + (o - 1);
                    const double zf = __hiloint2double(lane_bit(z[dp]) ? 0x40000000 : 0, 0);
                    acc = __builtin_fma(zf, h[dp], acc);
                }
                L[s] = acc;
            }
        };
        for (uint32_t first = 0; first < cnt[j]; first += K) {
            const uint32_t nrec = (cnt[j] - first) < (uint32_t)K ? cnt[j] - first : (uint32_t)K;
            const uint32_t sh = first == 0 ? shift[j] : stage_chunk(j, first, nrec);
            const double *hs = reinterpret_cast<const double *>(&stage[wib][j][sh]);
            const uint64_t *zq = reinterpret_cast<const uint64_t *>(
                g.rec_z + ((uint64_t)off[j] + first) * zstride + (uint64_t)lm.cb * D * 2);
            uint32_t k = 0;
            // two records per step: their scalar mask loads share one wait
            for (; k + 1 < nrec; k += 2) {
                record(hs + k * RP, zq + (uint64_t)k * (zstride / 2));
                record(hs + (k + 1) * RP, zq + (uint64_t)(k + 1) * (zstride / 2));
            }
            if (k < nrec) record(hs + k * RP, zq + (uint64_t)k * (zstride / 2));
        }
        newx[j] = draw_node<QM, UQ, EXP64>(L, qn, Wn[j] >> 8);
    }
    // the touch loads end here (their values are not used)
    asm volatile("" ::"v"(sink_z), "v"(sink_b));
    if (count && g.CB == 1) {
        uint32_t drawn = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) drawn |= (qnv[j] > 0 ? 1u : 0u) << j;
        count_quad<QM>(g.counts, quad, newx, qnv, drawn, cvalid, lane);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t node = quad * 4 + j;
            if (newx[j] >= 0 && cvalid) g.x[node * g.C + lm.c] = (uint8_t)newx[j];
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t node = quad * 4 + j;
        const bool nvalid = node < g.n && newx[j] >= 0;
        if (nvalid && cvalid) g.x[node * g.C + lm.c] = (uint8_t)newx[j];
        if (count) {
#pragma unroll
            for (int a = 0; a < QM; ++a) {
                const uint64_t bal = __ballot(nvalid && cvalid && newx[j] == a);
                if (nvalid && lane == 0 && a < qnv[j] && bal != 0)
                    atomicAdd(g.counts + node * QM + a, (uint32_t)__popcll(bal));
            }
        }
    }
}

// Counters of a node quad when each lane holds two chains (k_primal32):
// count_quad with the two chains' draws added.
template <int QM>
__device__ __forceinline__ void count_quad2(uint32_t *__restrict__ counts, int64_t quad,
                                            const int (&nx1)[4], const int (&nx2)[4],
                                            const int (&qn)[4], uint32_t drawn, bool ch1,
                                            bool ch2, int lane)
{
    uint32_t *cq = counts + quad * 4 * QM;
    uint32_t row = 0;
    uint64_t wmask = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const bool dj = (drawn >> j) & 1u;
#pragma unroll
        for (int a = 0; a < QM; ++a) {
            const uint32_t add = (uint32_t)__popcll(__ballot(dj && ch1 && nx1[j] == a)) +
                                 (uint32_t)__popcll(__ballot(dj && ch2 && nx2[j] == a));
            row = pdg_writelane_i32(cq[j * QM + a] + add, j * QM + a, row);
        }
        if (dj) wmask |= ((1ull << qn[j]) - 1ull) << (j * QM);
    }
    if (lane_bit(wmask)) cq[lane] = row;
}

// ---------------------------------------------------------------------------
// a4 + a5 with 17..32 chains: a wave takes one node quad; lane (g, l) is in
// record group g = lane / 16 and holds chains l and l + 16.  The four groups
// walk records k + g of the same node, so every h and mask word read from
// LDS serves two chains per lane (the LDS traffic per chain and entry is half
// that of one chain per lane, which bounded this kernel), and add their
// partial fields with a two-step butterfly before the draw (every group ends
// with the same sums).  The quad's records are walked as one stream of chunks
// (a chunk: up to K records of one node, their h values and 32-bit mask
// words); the next chunk is loaded into registers while the current one is
// read from the wave's LDS buffer, then written to the other buffer.
// ---------------------------------------------------------------------------
template <int QM, bool UQ, bool EXP64>
__global__ __launch_bounds__(256) void k_primal32(Graph g, uint32_t t, int count)
{
    sweep_args(g, t, count);
    constexpr int D = dim_d(QM);
    constexpr int RP = rec_len(QM);
    constexpr int G = 4;                                      // record groups per wave
    constexpr int BUF = 4864;                                 // LDS bytes per buffer (two per wave)
    constexpr int ZB = (4 * D + 15) / 16 * 16;                // zero mask block (once per wave)
    constexpr int K = (BUF - 32) / (8 * RP + 4 * D);          // records per chunk
    static_assert(K >= G, "chunk too small");
    constexpr int HB = (16 + 8 * RP * K + 15) / 16 * 16;      // h part of a buffer
    constexpr int NH = (HB + 1023) / 1024;                    // 16-byte loads per lane, h part
    constexpr int NZ = (16 + 4 * D * K + 1023) / 1024;        // and mask part
    __shared__ __align__(16) uint8_t lds[4][2 * BUF + ZB];
    const int lane = threadIdx.x & 63;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t quad = (int64_t)blockIdx.x * (blockDim.x >> 6) + wib;
    const int grp = lane >> 4;
    const int c1 = lane & 15, c2 = c1 + 16;
    const bool cv1 = c1 < g.C, cv2 = c2 < g.C;
    if (quad * 4 >= g.n) return;
    uint32_t off[4], cnt[4];
    uint32_t hub = 0;  // bit j: node j is a hub (drawn by the hub kernels)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        off[j] = g.inc_off[quad * 4 + j];
        cnt[j] = quad * 4 + j < g.n ? g.inc_cnt[quad * 4 + j] : 0u;
        if (g.heavy && cnt[j] > g.heavy) {
            hub |= 1u << j;
            cnt[j] = 0;
        }
    }
    uint8_t *reg = lds[wib];
    if (lane < ZB / 16)
        *reinterpret_cast<uint4 *>(reg + 2 * BUF + 16 * lane) = make_uint4(0, 0, 0, 0);
    const uint32_t *zero = reinterpret_cast<const uint32_t *>(reg + 2 * BUF);
    // rotating a mask word right by c + 2 puts chain c's bit at bit 30, the
    // one set bit of 2.0's high word
    const uint32_t rot1 = (uint32_t)(c1 + 2) & 31u, rot2 = (uint32_t)(c2 + 2) & 31u;
    auto sel = [&](const uint32_t (&a)[4], int j) -> uint32_t {
        return j == 0 ? a[0] : j == 1 ? a[1] : j == 2 ? a[2] : a[3];
    };
    auto skip_empty = [&](int &j, uint32_t &first) {
        while (j < 4 && first >= sel(cnt, j)) {
            ++j;
            first = 0;
        }
    };
    // registers of a chunk in flight
    uint4 rh[NH], rz[NZ];
    uint32_t sh_h = 0, sh_z = 0;  // byte shifts of its first record
    auto issue = [&](int j, uint32_t first) {
        const uint32_t nrec = min(sel(cnt, j) - first, (uint32_t)K);
        const uint64_t r0 = (uint64_t)sel(off, j) + first;
        const uint64_t ah = r0 * (RP * 8), az = r0 * (D * 4);
        sh_h = (uint32_t)(ah & 15);
        sh_z = (uint32_t)(az & 15);
        const uint8_t *ph = reinterpret_cast<const uint8_t *>(g.rec_p) + (ah - sh_h);
        const uint8_t *pz = reinterpret_cast<const uint8_t *>(g.rec_z) + (az - sh_z);
        const uint32_t bh = sh_h + nrec * (RP * 8), bz = sh_z + nrec * (D * 4);
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            const uint32_t o = (uint32_t)(i * 64 + lane) * 16;
            rh[i] = o < bh ? *reinterpret_cast<const uint4 *>(ph + o) : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < NZ; ++i) {
            const uint32_t o = (uint32_t)(i * 64 + lane) * 16;
            rz[i] = o < bz ? *reinterpret_cast<const uint4 *>(pz + o) : make_uint4(0, 0, 0, 0);
        }
    };
    auto commit = [&](int b) {  // registers -> LDS buffer b
        uint8_t *dst = reg + b * BUF;
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            const uint32_t o = (uint32_t)(i * 64 + lane) * 16;
            if (o < HB) *reinterpret_cast<uint4 *>(dst + o) = rh[i];
        }
#pragma unroll
        for (int i = 0; i < NZ; ++i) {
            const uint32_t o = (uint32_t)(i * 64 + lane) * 16;
            if (HB + o < BUF) *reinterpret_cast<uint4 *>(dst + HB + o) = rz[i];
        }
    };
    const Words wq1 = philox4x32_10((uint32_t)quad, (uint32_t)(quad >> 32),
                                    (kPhasePrimal << 30) | (uint32_t)c1, t, g.rk);
    const Words wq2 = philox4x32_10((uint32_t)quad, (uint32_t)(quad >> 32),
                                    (kPhasePrimal << 30) | (uint32_t)c2, t, g.rk);
    uint32_t drawn1 = 0, drawn2 = 0;  // byte j: 1 + the new state of node j (0: not drawn)
    double L1[QM], L2[QM];
    int j = 0;
    uint32_t first = 0;
    skip_empty(j, first);
    int jn = j;
    uint32_t fn = first;
    if (jn < 4) issue(jn, fn);
    int b = 0;
    int jdone = 0;  // nodes [0, jdone) are drawn
    auto word_of = [](const Words &w, int jj) {
        return (jj == 0 ? w.w0 : jj == 1 ? w.w1 : jj == 2 ? w.w2 : w.w3) >> 8;
    };
    auto draw_upto = [&](int jend) {  // draw record-less nodes below jend, in order
        for (; jdone < jend; ++jdone) {
            const int64_t node = quad * 4 + jdone;
            if (node >= g.n || ((hub >> jdone) & 1u)) continue;
            const int qn = UQ ? QM : (int)g.q[node];
            double Lb[QM];
#pragma unroll
            for (int a = 0; a < QM; ++a) Lb[a] = (UQ || a < qn) ? g.base[node * QM + a] : 0.0;
            drawn1 |= (uint32_t)(draw_node<QM, UQ, EXP64>(Lb, qn, word_of(wq1, jdone)) + 1) << (8 * jdone);
            drawn2 |= (uint32_t)(draw_node<QM, UQ, EXP64>(Lb, qn, word_of(wq2, jdone)) + 1) << (8 * jdone);
        }
    };
    while (jn < 4) {
        const uint32_t shh = sh_h, shz = sh_z;
        commit(b);
        const int jc = jn;
        const uint32_t fc = fn;
        const uint32_t nrec = min(sel(cnt, jc) - fc, (uint32_t)K);
        // next chunk in flight while this one is read
        fn = fc + nrec;
        skip_empty(jn, fn);
        if (jn < 4) issue(jn, fn);
        const int64_t node = quad * 4 + jc;
        const int qn = UQ ? QM : (int)g.q[node];
        if (fc == 0) {
            draw_upto(jc);  // record-less nodes before this one
            // group 0 starts from the node's base (lam and every c0), the others from 0
#pragma unroll
            for (int a = 0; a < QM; ++a) {
                L1[a] = (grp == 0 && (UQ || a < qn)) ? g.base[node * QM + a] : 0.0;
                L2[a] = L1[a];
            }
        }
        const double *hs = reinterpret_cast<const double *>(reg + b * BUF + shh);
        const uint32_t *zs = reinterpret_cast<const uint32_t *>(reg + b * BUF + HB + shz);
        for (uint32_t k = 0; k < nrec; k += G) {
            // group grp takes record k + grp; past the end it reads record k's h
            // with an all-zero mask, which adds nothing
            const bool has = k + grp < nrec;
            const double *h = hs + (has ? k + grp : k) * RP;
            const uint32_t *z = has ? zs + (k + grp) * D : zero;
#pragma unroll
            for (int s = 1; s < QM; ++s) {
                if (!UQ && s >= qn) break;
                double a1 = L1[s], a2 = L2[s];
#pragma unroll
                for (int o = 1; o < QM; ++o) {
                    const int dp = (s - 1) * (QM - 1) + (o - 1);
                    const uint32_t zw = z[dp];
                    const double hv = h[dp];
                    const uint32_t m1 = __builtin_amdgcn_alignbit(zw, zw, rot1) & 0x40000000u;
                    const uint32_t m2 = __builtin_amdgcn_alignbit(zw, zw, rot2) & 0x40000000u;
                    a1 = __builtin_fma(__hiloint2double((int)m1, 0), hv, a1);
                    a2 = __builtin_fma(__hiloint2double((int)m2, 0), hv, a2);
                }
                L1[s] = a1;
                L2[s] = a2;
            }
        }
        if (fc + nrec >= sel(cnt, jc)) {
            // groups g and g ^ 1, then pairs of groups: every group ends with the
            // same sums (IEEE addition is commutative)
#pragma unroll
            for (int s = 1; s < QM; ++s) {
                L1[s] += __shfl_xor(L1[s], 16);
                L2[s] += __shfl_xor(L2[s], 16);
            }
#pragma unroll
            for (int s = 1; s < QM; ++s) {
                L1[s] += __shfl_xor(L1[s], 32);
                L2[s] += __shfl_xor(L2[s], 32);
            }
            drawn1 |= (uint32_t)(draw_node<QM, UQ, EXP64>(L1, qn, word_of(wq1, jc)) + 1) << (8 * jc);
            drawn2 |= (uint32_t)(draw_node<QM, UQ, EXP64>(L2, qn, word_of(wq2, jc)) + 1) << (8 * jc);
            jdone = jc + 1;
        }
        b ^= 1;
    }
    draw_upto(4);
    int nx1[4], nx2[4];
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
        nx1[jj] = (int)((drawn1 >> (8 * jj)) & 255u) - 1;
        nx2[jj] = (int)((drawn2 >> (8 * jj)) & 255u) - 1;
    }
    int qnv[4];  // 0 for nodes this wave does not draw
#pragma unroll
    for (int jj = 0; jj < 4; ++jj)
        qnv[jj] = nx1[jj] >= 0 ? (UQ ? QM : (int)g.q[quad * 4 + jj]) : 0;
    const bool w1 = grp == 0 && cv1, w2 = grp == 0 && cv2;
    if (count) {
        // the wave owns the quad's counters (one chain block)
        uint32_t dmask = 0;
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) dmask |= (qnv[jj] > 0 ? 1u : 0u) << jj;
        count_quad2<QM>(g.counts, quad, nx1, nx2, qnv, dmask, w1, w2, lane);
    }
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
        const int64_t node = quad * 4 + jj;
        if (nx1[jj] >= 0 && w1) g.x[node * g.C + c1] = (uint8_t)nx1[jj];
        if (nx2[jj] >= 0 && w2) g.x[node * g.C + c2] = (uint8_t)nx2[jj];
    }
}

// ---------------------------------------------------------------------------
// Subset-sum tables of a record (chain-major dual words, zc_layout).  For own
// state r the field adds sum_o 2 theta_o h_ro over the other end's states o =
// 1..QM-1; byte r-1 of a chain's word holds those theta_o as bits o-1.  Per
// (record, r) the 16 sums over every subset of o = 1..4 (low nibble) and the
// 8 over o = 5..7 (bits 4..6) are tabulated once per wave, so a chain adds
// its field of state r with two table reads instead of QM-1 tests and FMAs.
// Table pair of (record k, own state r): 24 doubles at (k (QM-1) + r-1) 26.
// One lane writes a pair with twelve 16-byte stores; a stride of 26 doubles
// (52 dwords) puts the pairs of consecutive lanes in distinct LDS banks (at
// 24, every other lane hit the same banks and the stores were serialised).
// ---------------------------------------------------------------------------
constexpr int kZChunk = 4;  // records per step of the chain-major hub pieces
constexpr int kZPair = 26;  // doubles per (record, own state) table pair, 24 used

// One table pair from the 2 h of o = 1..QM-1 (entries past QM-1 zero):
// lo[m] = sum of the o = i+1 with bit i of m, i < 4; hi[m] likewise for o = i+5.
template <int QM>
__device__ __forceinline__ void build_tables(const double (&h)[QM - 1], double *__restrict__ dst)
{
    constexpr int S = QM - 1;
    const double a1 = 2.0 * h[0], a2 = 2.0 * h[1], a3 = 2.0 * h[2], a4 = 2.0 * h[3];
    const double b1 = S >= 5 ? 2.0 * h[S >= 5 ? 4 : 0] : 0.0;
    const double b2 = S >= 6 ? 2.0 * h[S >= 6 ? 5 : 0] : 0.0;
    const double b3 = S >= 7 ? 2.0 * h[S >= 7 ? 6 : 0] : 0.0;
    double T[24];
    T[0] = 0.0;
    T[1] = a1;
    T[2] = a2;
    T[3] = a2 + a1;
    T[4] = a3;
    T[5] = a3 + a1;
    T[6] = a3 + a2;
    T[7] = a3 + T[3];
#pragma unroll
    for (int m = 0; m < 8; ++m) T[8 + m] = m == 0 ? a4 : a4 + T[m];
    T[16] = 0.0;
    T[17] = b1;
    T[18] = b2;
    T[19] = b2 + b1;
    T[20] = b3;
    T[21] = b3 + b1;
    T[22] = b3 + b2;
    T[23] = b3 + T[19];
    double2 *d2 = reinterpret_cast<double2 *>(dst);
#pragma unroll
    for (int i = 0; i < 12; ++i) d2[i] = make_double2(T[2 * i], T[2 * i + 1]);
}

// Adds a chain's field of every own state r >= 1 of one record: L[r] += lo + hi
// of the table pair of (record, r) at the byte r-1 of its word w.
template <int QM>
__device__ __forceinline__ void add_tables(const double *__restrict__ tk, uint64_t w, double (&L)[QM])
{
    const uint32_t wl = (uint32_t)w, wh = (uint32_t)(w >> 32);
#pragma unroll
    for (int r = 1; r < QM; ++r) {
        const uint32_t src = r <= 4 ? wl : wh;
        const uint32_t sh = (uint32_t)(8 * ((r - 1) & 3));
        const uint32_t lo = __builtin_amdgcn_ubfe(src, sh, 4u), hi = __builtin_amdgcn_ubfe(src, sh + 4u, 3u);
        const double *t = tk + (r - 1) * kZPair;
        double a = L[r] + t[lo];
        L[r] = a + t[16 + hi];
    }
}

// ---------------------------------------------------------------------------
// a4 + a5 with 17..32 chains and q_max >= 6 (chain-major dual words): four
// nodes per wave, record group g = lane / 16 (chains l and l + 16 of lane l
// of the group) takes the node at position 4 Q + g of the node order (nodes
// sorted by record count, so the four take about as many steps; any order
// draws the same values) and walks its records, one per
// step, so a step takes up to four records, one per group.  A step's table
// pairs are built into the wave's LDS region by the first 4 (QM-1) lanes
// (lane (QM-1) g + r - 1 builds the pair of own state r of group g's record
// from the h row it loaded) and read back by the group's lanes.  Loads run
// through three register buffers, so while one step is processed the next
// two are in flight.  No cross-group sum is needed and the four nodes are drawn
// at once; a wave takes as many steps as its busiest node has records (in id
// order 1.36 times the mean over a quad on a Chung-Lu graph of mean degree 8;
// sorted, 1.00).
// ---------------------------------------------------------------------------
template <int QM, bool UQ, bool EXP64>
__global__ __launch_bounds__(256) void k_primal32z(Graph g, uint32_t t, int count)
{
    sweep_args(g, t, count);
    constexpr int D = dim_d(QM);
    constexpr int S = QM - 1;
    constexpr int G = 4;
    static_assert(G * S <= 64, "one table pair per lane");
    __shared__ __align__(16) double tab[4][G * S * kZPair];
    const int lane = threadIdx.x & 63;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t quad = (int64_t)blockIdx.x * (blockDim.x >> 6) + wib;
    const int grp = lane >> 4;
    const int c1 = lane & 15, c2 = c1 + 16;
    const bool cv1 = c1 < g.C, cv2 = c2 < g.C;
    if (quad * 4 >= g.n) return;
    // the wave's four nodes: positions 4 Q .. 4 Q + 3 of the node order (nodes
    // sorted by record count, so that they take about the same number of
    // steps) or of the ids; group g takes the node at position 4 Q + g
    uint32_t nd[4];
    bool vin[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t pos = quad * 4 + j;
        vin[j] = pos < g.n;
        nd[j] = vin[j] ? (g.order ? g.order[pos] : (uint32_t)pos) : 0u;
    }
    const int64_t node = grp == 0 ? nd[0] : grp == 1 ? nd[1] : grp == 2 ? nd[2] : nd[3];
    const bool nin = grp == 0 ? vin[0] : grp == 1 ? vin[1] : grp == 2 ? vin[2] : vin[3];
    const int kb = lane / S, rb = lane % S;  // builder: group kb, own state rb + 1
    const bool bl = lane < G * S;
    uint32_t cnt_g = 0, off_g = 0, cnt_b = 0, off_b = 0;
    bool hub_g = false;
    {
        uint32_t cnt[4], off[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            off[j] = g.inc_off[nd[j]];
            cnt[j] = vin[j] ? g.inc_cnt[nd[j]] : 0u;
            if (g.heavy && cnt[j] > g.heavy) {
                if (j == grp) hub_g = true;
                cnt[j] = 0;
            }
        }
        cnt_g = grp == 0 ? cnt[0] : grp == 1 ? cnt[1] : grp == 2 ? cnt[2] : cnt[3];
        off_g = grp == 0 ? off[0] : grp == 1 ? off[1] : grp == 2 ? off[2] : off[3];
        cnt_b = kb == 0 ? cnt[0] : kb == 1 ? cnt[1] : kb == 2 ? cnt[2] : kb == 3 ? cnt[3] : 0u;
        off_b = kb == 0 ? off[0] : kb == 1 ? off[1] : kb == 2 ? off[2] : kb == 3 ? off[3] : 0u;
    }
    // steps of the wave: the largest record count of its nodes
    uint32_t nsteps = cnt_g;
#pragma unroll
    for (int o = 16; o < 64; o <<= 1) nsteps = max(nsteps, (uint32_t)__shfl_xor((int)nsteps, o));
    nsteps = __builtin_amdgcn_readfirstlane(nsteps);
    double *tw = tab[wib];
    const uint64_t *z64 = reinterpret_cast<const uint64_t *>(g.rec_z);
    const uint64_t C = (uint64_t)g.C;
    // loads are unconditional and raw (lanes without a record read the
    // pool's first one); the predicates are applied where the values are used,
    // so nothing waits on a load before its step and the later steps' loads
    // stay in flight
    const int cz2 = cv2 ? c2 : c1;
    auto issue = [&](uint32_t st, double (&h)[S], uint64_t &w1, uint64_t &w2) {
        const bool hb = bl && st < cnt_b;
        const double *hp = g.rec_p + (hb ? ((uint64_t)off_b + st) * D + rb * S : 0ull);
#pragma unroll
        for (int o = 0; o < S; ++o) h[o] = hp[o];
        const uint64_t r = st < cnt_g ? (uint64_t)off_g + st : 0ull;
        w1 = z64[r * C + c1];
        w2 = z64[r * C + cz2];
    };
    const int qn = UQ ? QM : (nin ? (int)g.q[node] : QM);
    double L1[QM], L2[QM];
#pragma unroll
    for (int a = 0; a < QM; ++a) {
        L1[a] = (nin && (UQ || a < qn)) ? g.base[node * QM + a] : 0.0;
        L2[a] = L1[a];
    }
    auto process = [&](uint32_t st, const double (&hc)[S], uint64_t wc1, uint64_t wc2) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (bl && st < cnt_b) build_tables<QM>(hc, tw + (kb * S + rb) * kZPair);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // a group whose node has no record at this step reads its table pair
        // at index 0 (0.0) with a zero word; those tables were built at an
        // earlier step or hold the zeros written below
        const bool has = st < cnt_g;
        const double *tk = tw + grp * (S * kZPair);
        add_tables<QM>(tk, has ? wc1 : 0ull, L1);
        asm volatile("" ::: "memory");
        add_tables<QM>(tk, has && cv2 ? wc2 : 0ull, L2);
        asm volatile("" ::: "memory");
    };
    // table pairs of groups without a record at some step are read at index
    // 0: make every pair's entries 0 and 16 zero once
    if (bl) {
        tw[(kb * S + rb) * kZPair] = 0.0;
        tw[(kb * S + rb) * kZPair + 16] = 0.0;
    }
    double hA[S], hB[S], hC[S];
    uint64_t wA1, wA2, wB1, wB2, wC1, wC2;
    if (0 < nsteps) issue(0, hA, wA1, wA2);
    if (1 < nsteps) issue(1, hB, wB1, wB2);
    if (2 < nsteps) issue(2, hC, wC1, wC2);
    for (uint32_t st = 0; st < nsteps; st += 3) {
        process(st, hA, wA1, wA2);
        if (st + 3 < nsteps) issue(st + 3, hA, wA1, wA2);
        if (st + 1 >= nsteps) break;
        process(st + 1, hB, wB1, wB2);
        if (st + 4 < nsteps) issue(st + 4, hB, wB1, wB2);
        if (st + 2 >= nsteps) break;
        process(st + 2, hC, wC1, wC2);
        if (st + 5 < nsteps) issue(st + 5, hC, wC1, wC2);
    }
    // draw: a node i is drawn with word i mod 4 of its chains' calls on the
    // node quad i / 4, wherever the order puts it
    const uint32_t nq = (uint32_t)(node >> 2);
    const Words wq1 = philox4x32_10(nq, 0u, (kPhasePrimal << 30) | (uint32_t)c1, t, g.rk);
    const Words wq2 = philox4x32_10(nq, 0u, (kPhasePrimal << 30) | (uint32_t)c2, t, g.rk);
    const bool drawn = nin && !hub_g;
    const int nx1 = draw_node<QM, UQ, EXP64>(L1, qn, word_at(wq1, (int)(node & 3)) >> 8);
    const int nx2 = draw_node<QM, UQ, EXP64>(L2, qn, word_at(wq2, (int)(node & 3)) >> 8);
    if (drawn && cv1) g.x[node * g.C + c1] = (uint8_t)nx1;
    if (drawn && cv2) g.x[node * g.C + c2] = (uint8_t)nx2;
    if (count) {
        // the wave owns its nodes' counters (one chain block): lane a of a
        // group adds the group's draws of state a to its node's counter a
        const uint32_t gsh = 16u * (uint32_t)grp;
        uint32_t add = 0;
#pragma unroll
        for (int a = 0; a < QM; ++a) {
            const uint64_t b1 = __ballot(drawn && cv1 && nx1 == a);
            const uint64_t b2 = __ballot(drawn && cv2 && nx2 == a);
            const uint32_t na = (uint32_t)__popc((uint32_t)(b1 >> gsh) & 0xFFFFu) +
                                (uint32_t)__popc((uint32_t)(b2 >> gsh) & 0xFFFFu);
            if (c1 == a) add = na;
        }
        // (an add without return: nothing waits on it; the wave owns the counter)
        if (drawn && c1 < qn && add != 0u) atomicAdd(g.counts + node * QM + c1, add);
    }
}

// ---------------------------------------------------------------------------
// a4 for hubs.  A node with more than kHubThreshold incidence entries is a
// hub: the quad kernels skip it, and its records are split into pieces of at
// most kHubPiece so that one hub's work spreads over many waves.
// k_hub_pieces: one wave per (piece, chain block) sums sum_records sum_o
// 2 theta h over the piece (records staged in the wave's LDS region, the
// chain's mask bit tested as in k_primal32); with LPI <= 32 the 64 / LPI lane
// groups take consecutive records of a step and are added at the end by a
// butterfly (every lane ends with its chain's total, the same in every group).
// The partial field goes to part[((piece * CB + cb) * (QM - 1) + s - 1) * 64 + lane].
// k_hub_finish: one wave per (hub, chain block) adds the node's base and its
// pieces' partial fields in piece order, then draws, stores x and counts.
// ---------------------------------------------------------------------------
constexpr uint32_t kHubThreshold = 256;
constexpr uint32_t kHubPiece = 128;

template <int QM, int LPI>
__global__ __launch_bounds__(256) void k_hub_pieces(Graph g, int64_t np,
                                                    const uint32_t *__restrict__ pnode,
                                                    const uint32_t *__restrict__ pfirst,
                                                    const uint32_t *__restrict__ pn,
                                                    double *__restrict__ part)
{
    constexpr int D = dim_d(QM);
    constexpr int RP = rec_len(QM);
    constexpr int BUF = 4096;                   // LDS bytes per wave
    constexpr int ZB = (8 * D + 15) / 16 * 16;  // zero mask block
    constexpr int NLD = BUF / 1024;
    __shared__ __align__(16) uint8_t lds[4][BUF];
    const int lane = threadIdx.x & 63;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + wib;
    const int CB = g.CB;
    const int64_t piece = w / CB;
    const int cb = (int)(w - piece * CB);
    if (piece >= np) return;
    const uint32_t node = pnode[piece];
    const uint64_t r0 = (uint64_t)g.inc_off[node] + pfirst[piece];
    const uint32_t n = pn[piece];
    const int p = LPI == 64 ? 0 : lane / LPI;
    constexpr uint32_t PR = LPI == 64 ? 1u : 64u / LPI;             // records per step
    const uint32_t zr = LPI == 64 ? 2u * D * (uint32_t)CB : (uint32_t)D;  // u32 words per record
    const uint32_t zsel = LPI == 64 ? (uint32_t)(cb * 2 * D + (lane >> 5)) : 0u;
    constexpr uint32_t ZSTEP = LPI == 64 ? 2u : 1u;
    const uint32_t cbit = LPI == 64 ? (uint32_t)(lane & 31) : (uint32_t)(lane % LPI);
    const uint32_t rot = (cbit + 2u) & 31u;
    const uint32_t K = (uint32_t)(BUF - ZB - 48) / (uint32_t)(RP * 8 + 4 * zr);
    const uint32_t HB = (16 + K * (RP * 8) + 15) & ~15u;
    uint8_t *reg = lds[wib];
    if (lane < ZB / 16)
        *reinterpret_cast<uint4 *>(reg + BUF - ZB + 16 * lane) = make_uint4(0, 0, 0, 0);
    const uint32_t *zero = reinterpret_cast<const uint32_t *>(reg + BUF - ZB);
    double L[QM];
#pragma unroll
    for (int a = 0; a < QM; ++a) L[a] = 0.0;
    for (uint32_t first = 0; first < n; first += K) {
        const uint32_t nrec = min(n - first, K);
        // the chunk's h rows (to 0) and mask words (to HB) in 16-byte aligned
        // pieces: every lane loads its pieces of both without a branch (pieces
        // past the end re-read the first, which lies in the chunk's first
        // record) and writes them, a piece past the end to the first piece's
        // place with the first piece's bytes, so no load is moved into a
        // branch and all of a chunk's loads share one wait
        const uint64_t ah = (r0 + first) * (RP * 8), az = (r0 + first) * zr * 4;
        const uint64_t ah16 = ah & ~(uint64_t)15, az16 = az & ~(uint64_t)15;
        const uint32_t sh = (uint32_t)(ah - ah16), sz = (uint32_t)(az - az16);
        const uint32_t bh = sh + nrec * (RP * 8), bz = sz + nrec * zr * 4;
        const uint8_t *ph = reinterpret_cast<const uint8_t *>(g.rec_p) + ah16;
        const uint8_t *pz = reinterpret_cast<const uint8_t *>(g.rec_z) + az16;
        uint4 vh[NLD], vz[NLD];
#pragma unroll
        for (int i = 0; i < NLD; ++i) {
            const uint32_t o = (uint32_t)(i * 64 + lane) * 16;
            vh[i] = *reinterpret_cast<const uint4 *>(ph + (o < bh ? o : 0u));
            vz[i] = *reinterpret_cast<const uint4 *>(pz + (o < bz ? o : 0u));
        }
#pragma unroll
        for (int i = 0; i < NLD; ++i) {
            const uint32_t o = (uint32_t)(i * 64 + lane) * 16;
            *reinterpret_cast<uint4 *>(reg + (o < bh ? o : 0u)) = vh[i];
            *reinterpret_cast<uint4 *>(reg + HB + (o < bz ? o : 0u)) = vz[i];
        }
        const double *hs = reinterpret_cast<const double *>(reg + sh);
        const uint32_t *zs = reinterpret_cast<const uint32_t *>(reg + HB + sz);
        for (uint32_t k = 0; k < nrec; k += PR) {
            // lane group p takes record k + p; past the end it reads record
            // k's h with an all-zero mask, which adds nothing
            const bool has = k + p < nrec;
            const double *h = hs + (has ? k + p : k) * RP;
            const uint32_t *z = has ? zs + (k + p) * zr + zsel : zero;
#pragma unroll
            for (int s = 1; s < QM; ++s) {
                double acc = L[s];
#pragma unroll
                for (int o = 1; o < QM; ++o) {
                    const int dp = (s - 1) * (QM - 1) + (o - 1);
                    const uint32_t wz = z[dp * ZSTEP];
                    const uint32_t hi = __builtin_amdgcn_alignbit(wz, wz, rot) & 0x40000000u;
                    acc = __builtin_fma(__hiloint2double((int)hi, 0), h[dp], acc);
                }
                L[s] = acc;
            }
        }
    }
#pragma unroll
    for (int sh = 32; sh >= LPI && sh > 0; sh >>= 1) {
#pragma unroll
        for (int s = 1; s < QM; ++s) L[s] += __shfl_xor(L[s], sh);
    }
#pragma unroll
    for (int s = 1; s < QM; ++s)
        part[((piece * CB + cb) * (QM - 1) + (s - 1)) * 64 + lane] = L[s];
}

// k_hub_pieces for chain-major dual words (17..32 chains, q_max >= 6): one
// wave per piece, lanes, tables and the two chunk buffers as in k_primal32z;
// the piece's partial field of chain l % 32 goes to lane l of its rows of
// part (as k_hub_finish with 32 chains per item reads it).
template <int QM>
__global__ __launch_bounds__(256) void k_hub_pieces_z(Graph g, int64_t np,
                                                      const uint32_t *__restrict__ pnode,
                                                      const uint32_t *__restrict__ pfirst,
                                                      const uint32_t *__restrict__ pn,
                                                      double *__restrict__ part)
{
    constexpr int D = dim_d(QM);
    constexpr int S = QM - 1;
    constexpr int G = 4;
    constexpr int K = kZChunk;
    constexpr int KG = K / G;
    __shared__ __align__(16) double tab[4][K * S * kZPair];
    const int lane = threadIdx.x & 63;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t piece = (int64_t)blockIdx.x * (blockDim.x >> 6) + wib;
    if (piece >= np) return;
    const int grp = lane >> 4;
    const int c1 = lane & 15, c2 = c1 + 16;  // c1 < 17 <= C: always a chain
    const bool cv2 = c2 < g.C;
    const uint32_t node = pnode[piece];
    const uint64_t rbase = (uint64_t)g.inc_off[node] + pfirst[piece];
    const uint32_t n = pn[piece];
    double *tw = tab[wib];
    const int kb = lane / S, rb = lane % S;
    const bool bl = lane < K * S;
    const uint64_t *z64 = reinterpret_cast<const uint64_t *>(g.rec_z);
    const uint64_t C = (uint64_t)g.C;
    // unconditional raw loads, predicates applied at use (as in k_primal32z)
    const int cz2 = cv2 ? c2 : c1;
    auto issue = [&](uint32_t first, double (&h)[S], uint64_t (&w1)[KG], uint64_t (&w2)[KG]) {
        const uint32_t nrec = min(n - first, (uint32_t)K);
        const uint64_t r0 = rbase + first;
        const bool hb = bl && (uint32_t)kb < nrec;
        const double *hp = g.rec_p + (hb ? (r0 + (uint64_t)kb) * D + rb * S : 0ull);
#pragma unroll
        for (int o = 0; o < S; ++o) h[o] = hp[o];
#pragma unroll
        for (int i = 0; i < KG; ++i) {
            const uint32_t k = (uint32_t)(grp + G * i);
            const uint64_t r = k < nrec ? r0 + k : 0ull;
            w1[i] = z64[r * C + c1];
            w2[i] = z64[r * C + cz2];
        }
    };
    double L1[QM], L2[QM];
#pragma unroll
    for (int a = 0; a < QM; ++a) L1[a] = L2[a] = 0.0;
    auto process = [&](uint32_t first, const double (&hc)[S], const uint64_t (&wc1)[KG],
                       const uint64_t (&wc2)[KG]) {
        const uint32_t nrec = min(n - first, (uint32_t)K);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (bl && (uint32_t)kb < nrec) build_tables<QM>(hc, tw + (kb * S + rb) * kZPair);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int i = 0; i < KG; ++i) {
            const uint32_t k = (uint32_t)(grp + G * i);
            const bool has = k < nrec;
            const double *tk = tw + (has ? k : 0u) * (S * kZPair);
            add_tables<QM>(tk, has ? wc1[i] : 0ull, L1);
            asm volatile("" ::: "memory");
            add_tables<QM>(tk, has && cv2 ? wc2[i] : 0ull, L2);
            asm volatile("" ::: "memory");
        }
    };
    double hA[S], hB[S];
    uint64_t wA1[KG], wA2[KG], wB1[KG], wB2[KG];
    uint32_t fA = 0, fB = K;  // first record of the chunk in each buffer
    if (fA < n) issue(fA, hA, wA1, wA2);
    if (fB < n) issue(fB, hB, wB1, wB2);
    while (fA < n) {
        process(fA, hA, wA1, wA2);
        fA += 2 * K;
        if (fA < n) issue(fA, hA, wA1, wA2);
        if (fB >= n) break;
        process(fB, hB, wB1, wB2);
        fB += 2 * K;
        if (fB < n) issue(fB, hB, wB1, wB2);
    }
#pragma unroll
    for (int s = 1; s < QM; ++s) {
        L1[s] += __shfl_xor(L1[s], 16);
        L2[s] += __shfl_xor(L2[s], 16);
    }
#pragma unroll
    for (int s = 1; s < QM; ++s) {
        L1[s] += __shfl_xor(L1[s], 32);
        L2[s] += __shfl_xor(L2[s], 32);
    }
#pragma unroll
    for (int s = 1; s < QM; ++s)
        part[(piece * (QM - 1) + (s - 1)) * 64 + lane] = (lane & 16) ? L2[s] : L1[s];
}

template <int QM, bool UQ, bool EXP64, int LPI>
__global__ __launch_bounds__(256) void k_hub_finish(Graph g, int64_t nh,
                                                    const uint32_t *__restrict__ hnode,
                                                    const uint32_t *__restrict__ hpfirst,
                                                    const double *__restrict__ part, uint32_t t,
                                                    int count)
{
    sweep_args(g, t, count);
    const int lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) +
                      __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int CB = g.CB;
    const int64_t k = w / CB;
    const int cb = (int)(w - k * CB);
    if (k >= nh) return;
    const uint64_t node = hnode[k];
    const int c = LPI == 64 ? cb * 64 + lane : lane % LPI;
    const bool cvalid = c < g.C && (LPI == 64 || lane < LPI);
    const int qn = UQ ? QM : (int)g.q[node];
    double L[QM];
#pragma unroll
    for (int a = 0; a < QM; ++a) L[a] = (UQ || a < qn) ? g.base[node * QM + a] : 0.0;
    for (uint32_t pc = hpfirst[k]; pc < hpfirst[k + 1]; ++pc) {
#pragma unroll
        for (int s = 1; s < QM; ++s)
            if (UQ || s < qn) L[s] += part[(((int64_t)pc * CB + cb) * (QM - 1) + (s - 1)) * 64 + lane];
    }
    // the node's word of its quad's call, as the quad kernels draw it
    const uint64_t quad = node >> 2;
    const Words wq = philox4x32_10((uint32_t)quad, (uint32_t)(quad >> 32),
                                   (kPhasePrimal << 30) | (uint32_t)c, t, g.rk);
    const uint32_t U = word_at(wq, (int)(node & 3)) >> 8;
    const int xn = draw_node<QM, UQ, EXP64>(L, qn, U);
    if (cvalid) g.x[node * g.C + c] = (uint8_t)xn;
    if (count) {
#pragma unroll
        for (int a = 0; a < QM; ++a) {
            const uint64_t bal = __ballot(cvalid && xn == a);
            if (lane == 0 && a < qn && bal != 0) {
                if (CB == 1)  // this wave owns the node's counters
                    g.counts[node * QM + a] += (uint32_t)__popcll(bal);
                else
                    atomicAdd(g.counts + node * QM + a, (uint32_t)__popcll(bal));
            }
        }
    }
}

// ---------------------------------------------------------------------------
// a4 + a5: primal phase and marginal counting.  Lane (node quad Q, chain c)
// takes one generator call (Q, PRIMAL, c, t) and walks the quad's four nodes;
// node 4Q + j draws with word j.  For node i:
//   L(a) = lam(a) + sum over the node's incidence records of the field of a:
//   src side c0_row(a) + sum_b 2 theta_ab h_ab, dst side c0_col(b) + sum_a 2 theta_ab |h_ab|;
// a record is stored in the node's own orientation (row = the node's state),
// so both sides read the same way; padded entries and tombstones are zero.
// Then the categorical draw of draw_node.  This generic form serves up to 16
// chains (64 / LPI quads per wave, per-lane record loads): the one-launch
// sweeps of small graphs, and full launches with one chain or binary records;
// k_primal_st is the same arithmetic for 8 or 16 chains and larger records,
// k_primal64 and k_primal32 the shapes for more chains.
// ---------------------------------------------------------------------------
template <int QM, int LPI, bool UQ, bool EXP64>
__device__ __forceinline__ void primal_wave(const Graph &g, uint32_t t, int count,
                                            const LaneMap<LPI> lm)
{
    static_assert(LPI <= 16, "33 or more chains: k_primal64; 17..32: k_primal32");
    constexpr int D = dim_d(QM);
    constexpr int RP = rec_len(QM);
    const int64_t quad = lm.item;
    const bool cvalid = lm.c < g.C;
    const Words wq = philox4x32_10((uint32_t)quad, (uint32_t)(quad >> 32),
                                   (kPhasePrimal << 30) | (uint32_t)lm.c, t, g.rk);
    const uint32_t Wn[4] = {wq.w0, wq.w1, wq.w2, wq.w3};
    // segment table of the quad (the arrays are padded to a multiple of four
    // nodes; entries past n are zero)
    uint32_t off[4] = {0, 0, 0, 0}, cnt[4] = {0, 0, 0, 0};
    uint32_t hub = 0;  // bit j: node j is a hub (drawn by the hub kernels)
    if (quad * 4 < g.n) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            off[j] = g.inc_off[quad * 4 + j];
            cnt[j] = g.inc_cnt[quad * 4 + j];
            if (g.heavy && cnt[j] > g.heavy) hub |= 1u << j;
        }
    }
    int newx[4], qnv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t node = quad * 4 + j;
        newx[j] = -1;
        qnv[j] = 0;
        if (node >= g.n || ((hub >> j) & 1u)) continue;
        const int qn = UQ ? QM : (int)g.q[node];
        qnv[j] = qn;
        // the theta-free part (lam and every c0) is the node's base
        double L[QM];
#pragma unroll
        for (int a = 0; a < QM; ++a) L[a] = (UQ || a < qn) ? g.base[node * QM + a] : 0.0;
        const double *hp = g.rec_p + (uint64_t)off[j] * RP;
        const uint32_t *zp = g.rec_z + (uint64_t)off[j] * D;
        auto add_record = [&](const double (&h)[D], const uint32_t (&z)[D]) {
#pragma unroll
            for (int s = 1; s < QM; ++s) {
                if (!UQ && s >= qn) break;
                double acc = L[s];
#pragma unroll
                for (int o = 1; o < QM; ++o) {
                    // acc + 2 theta h in one FMA: the factor is 0.0 or 2.0 and 2 h is exact
                    const int dp = (s - 1) * (QM - 1) + (o - 1);
                    const bool th = ((z[dp] >> (lm.c & 31)) & 1u) != 0;
                    acc = __builtin_fma(__hiloint2double(th ? 0x40000000 : 0, 0), h[dp], acc);
                }
                L[s] = acc;
            }
        };
        if constexpr (D <= 9) {
            // two records per step, both loaded before either is added (the
            // second index stays on the last record past the end), so a lane
            // waits once per two records; the sums keep record order
            for (uint32_t k = 0; k < cnt[j]; k += 2) {
                const uint32_t k1 = k + 1 < cnt[j] ? k + 1 : k;
                double h0[D], h1[D];
                uint32_t z0[D], z1[D];
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    h0[d] = hp[(uint64_t)k * RP + d];
                    z0[d] = zp[(uint64_t)k * D + d];
                    h1[d] = hp[(uint64_t)k1 * RP + d];
                    z1[d] = zp[(uint64_t)k1 * D + d];
                }
                add_record(h0, z0);
                if (k + 1 < cnt[j]) add_record(h1, z1);
            }
        } else {
            for (uint32_t k = 0; k < cnt[j]; ++k, hp += RP, zp += D) {
#pragma unroll
                for (int s = 1; s < QM; ++s) {
                    if (!UQ && s >= qn) break;
                    double acc = L[s];
#pragma unroll
                    for (int o = 1; o < QM; ++o) {
                        const int dp = (s - 1) * (QM - 1) + (o - 1);
                        const bool th = ((zp[dp] >> (lm.c & 31)) & 1u) != 0;
                        acc = __builtin_fma(__hiloint2double(th ? 0x40000000 : 0, 0), hp[dp], acc);
                    }
                    L[s] = acc;
                }
            }
        }
        newx[j] = draw_node<QM, UQ, EXP64>(L, qn, Wn[j] >> 8);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t node = quad * 4 + j;
        const bool nvalid = node < g.n && !((hub >> j) & 1u);
        const bool active = nvalid && cvalid;
        if (active) g.x[node * g.C + lm.c] = (uint8_t)newx[j];
        if (count) {
            // one chain block: the lane group of the quad owns the node's
            // counters (adds without return, so nothing waits on them)
            const bool leader = nvalid && (lm.lane % LPI == 0);
            const int p0 = (lm.lane / LPI) * LPI;
#pragma unroll
            for (int a = 0; a < QM; ++a) {
                const uint64_t mine =
                    (__ballot(active && newx[j] == a) >> p0) & ((1ull << LPI) - 1ull);
                if (leader && a < qnv[j] && mine != 0)
                    atomicAdd(g.counts + node * QM + a, (uint32_t)__popcll(mine));
            }
        }
    }
}

template <int QM, int LPI, bool UQ, bool EXP64>
__global__ __launch_bounds__(256) void k_primal(Graph g, uint32_t t, int count)
{
    sweep_args(g, t, count);
    primal_wave<QM, LPI, UQ, EXP64>(g, t, count, LaneMap<LPI>(g.C));
}

// ---------------------------------------------------------------------------
// a4 + a5 with 8 or 16 chains per item on full launches: primal_wave's
// arithmetic with each record loaded once per wave.  In primal_wave the LPI
// lanes of an item all load the same words, so every load instruction moves
// each byte LPI times.  Here step k of node j takes record k of node j of each
// of the wave's P quads: its P h rows (D doubles) and P mask rows (D words) are
// spread over the lanes, element e = 64 i + lane being entry e mod D of quad
// e / D, loaded by one lane, written to the wave's LDS region (rows padded to
// D + 1 elements, so the rows that one read touches fall in distinct banks) and
// read back by the item's lanes as broadcasts.  The next step's elements are
// loaded before the current step is summed.  The sums run in primal_wave's
// order (records in order, entries in order), so states and counts are those
// of primal_wave bit for bit.
// ---------------------------------------------------------------------------
// Uniform q up to 5: at most 80 VGPRs (six waves per SIMD) without spills.
template <int QM, int LPI, bool UQ, bool EXP64>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(UQ && QM <= 5 ? 6 : 1))) void k_primal_st(
    Graph g, uint32_t t, int count)
{
    static_assert(LPI == 8 || LPI == 16, "staged generic primal: 8 or 16 chains per item");
    sweep_args(g, t, count);
    constexpr int D = dim_d(QM);
    static_assert(rec_len(QM) == D, "one h per entry");
    constexpr int P = 64 / LPI;      // quads per wave
    constexpr int SH = D + 1;        // LDS row stride (elements)
    constexpr int NE = P * D;        // elements per step
    constexpr int NL = (NE + 63) / 64;
    __shared__ double lh[4][P * SH];
    __shared__ uint32_t lz[4][P * SH];
    const LaneMap<LPI> lm(g.C);
    const int lane = lm.lane;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    double *wh = lh[wib];
    uint32_t *wz = lz[wib];
    const int64_t quad = lm.item;
    const int p = lane / LPI;
    const bool cvalid = lm.c < g.C;
    const Words wq = philox4x32_10((uint32_t)quad, (uint32_t)(quad >> 32),
                                   (kPhasePrimal << 30) | (uint32_t)lm.c, t, g.rk);
    const uint32_t Wn[4] = {wq.w0, wq.w1, wq.w2, wq.w3};
    uint32_t off[4] = {0, 0, 0, 0}, cnt[4] = {0, 0, 0, 0};
    uint32_t hub = 0;  // bit j: node j is a hub (drawn by the hub kernels)
    if (quad * 4 < g.n) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            off[j] = g.inc_off[quad * 4 + j];
            cnt[j] = g.inc_cnt[quad * 4 + j];
            if (g.heavy && cnt[j] > g.heavy) {
                hub |= 1u << j;
                cnt[j] = 0;
            }
        }
    }
    // element e = 64 i + lane of a step: entry ede of quad epe (-1: none)
    int epe[NL], ede[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        const int e = 64 * i + lane;
        epe[i] = e < NE ? e / D : -1;
        ede[i] = e < NE ? e - (e / D) * D : 0;
    }
    int newx[4], qnv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t node = quad * 4 + j;
        const bool drawn = node < g.n && !((hub >> j) & 1u);
        const int qn = UQ ? QM : (drawn ? (int)g.q[node] : 0);
        newx[j] = -1;
        qnv[j] = 0;
        // the base row is read by every lane (node 0's when the node is not
        // drawn) and selected where it is used, so no load waits on a branch
        double L[QM];
        const int64_t nb = drawn ? node : 0;
#pragma unroll
        for (int a = 0; a < QM; ++a) {
            const double b = g.base[nb * QM + a];
            L[a] = (drawn && (UQ || a < qn)) ? b : 0.0;
        }
        // each element's record index (in elements) and record count, from
        // the lanes of its quad
        uint64_t eb[NL];
        uint32_t ec[NL];
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int from = (epe[i] < 0 ? 0 : epe[i]) * LPI;
            const uint32_t o = (uint32_t)__shfl((int)off[j], from);
            const uint32_t n = (uint32_t)__shfl((int)cnt[j], from);
            eb[i] = (uint64_t)o * D + (uint64_t)ede[i];
            ec[i] = epe[i] < 0 ? 0u : n;
        }
        const uint32_t mine = cnt[j];  // records of this lane's node j (0: hub, padding)
        // Elements of step k, loaded unconditionally (an element without a
        // record at step k reads element 0; no lane reads its row), into two
        // buffers used in turn, so that step k + 1's loads stay in flight
        // while step k is summed.  Only when some quad of the wave has a
        // record: a context without edges has no record arrays.
        auto issue = [&](uint32_t k, double (&vh)[NL], uint32_t (&vz)[NL]) {
#pragma unroll
            for (int i = 0; i < NL; ++i) {
                const uint64_t e = k < ec[i] ? eb[i] + (uint64_t)k * D : 0ull;
                vh[i] = g.rec_p[e];
                vz[i] = g.rec_z[e];
            }
        };
        auto step = [&](uint32_t k, const double (&vh)[NL], const uint32_t (&vz)[NL]) {
            // the previous step's reads are issued before these writes (LDS
            // operations of a wave complete in order)
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int i = 0; i < NL; ++i) {
                if (epe[i] >= 0) {
                    wh[epe[i] * SH + ede[i]] = vh[i];
                    wz[epe[i] * SH + ede[i]] = vz[i];
                }
            }
            __builtin_amdgcn_wave_barrier();
            if (k < mine) {
                const double *h = wh + p * SH;
                const uint32_t *z = wz + p * SH;
#pragma unroll
                for (int s = 1; s < QM; ++s) {
                    if (!UQ && s >= qn) break;
                    double acc = L[s];
#pragma unroll
                    for (int o = 1; o < QM; ++o) {
                        // acc + 2 theta h in one FMA: the factor is 0.0 or 2.0 and 2 h is exact
                        const int dp = (s - 1) * (QM - 1) + (o - 1);
                        const bool th = ((z[dp] >> (lm.c & 31)) & 1u) != 0;
                        acc = __builtin_fma(__hiloint2double(th ? 0x40000000 : 0, 0), h[dp], acc);
                    }
                    L[s] = acc;
                }
            }
        };
        if (__ballot(0u < mine) != 0) {
            double ha[NL], hb[NL];
            uint32_t za[NL], zb[NL];
            issue(0, ha, za);
            for (uint32_t k = 0;; k += 2) {
                issue(k + 1, hb, zb);
                step(k, ha, za);
                if (__ballot(k + 1 < mine) == 0) break;
                issue(k + 2, ha, za);
                step(k + 1, hb, zb);
                if (__ballot(k + 2 < mine) == 0) break;
            }
        }
        if (drawn) {
            qnv[j] = qn;
            newx[j] = draw_node<QM, UQ, EXP64>(L, qn, Wn[j] >> 8);
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t node = quad * 4 + j;
        const bool nvalid = node < g.n && !((hub >> j) & 1u);
        const bool active = nvalid && cvalid;
        if (active) g.x[node * g.C + lm.c] = (uint8_t)newx[j];
        if (count) {
            // one chain block: the lane group of the quad owns the node's
            // counters (adds without return, so nothing waits on them)
            const bool leader = nvalid && (lane % LPI == 0);
            const int p0 = p * LPI;
#pragma unroll
            for (int a = 0; a < QM; ++a) {
                const uint64_t mine =
                    (__ballot(active && newx[j] == a) >> p0) & ((1ull << LPI) - 1ull);
                if (leader && a < qnv[j] && mine != 0)
                    atomicAdd(g.counts + node * QM + a, (uint32_t)__popcll(mine));
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Many sweeps of a small graph in one launch (up to 16 chains): one work-group
// whose waves take the dual waves of a sweep in turn, meet at a barrier, take
// the primal waves, and meet again.  The per-wave work is that of k_dual and
// k_primal, so the trajectory is the one separate launches give; what goes
// away is the launch latency, which bounds small graphs.  Sweeps t0 + 1 ..
// t0 + n; counting from sweep burn_in + 1.
// ---------------------------------------------------------------------------
template <int QM, int LPI, bool UQ, bool EXP64>
__global__ __launch_bounds__(1024) void k_sweeps(Graph g, uint32_t t0, int32_t n,
                                                 int64_t burn_in, int64_t dual_waves,
                                                 int64_t primal_waves)
{
    const int64_t w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nw = blockDim.x >> 6;
    for (int32_t s = 0; s < n; ++s) {
        const uint32_t t = t0 + 1u + (uint32_t)s;
        for (int64_t v = w; v < dual_waves; v += nw)
            dual_wave<QM, LPI, UQ>(g, t, LaneMap<LPI>(g.C, v));
        __syncthreads();
        const int count = (int64_t)t > burn_in ? 1 : 0;
        for (int64_t v = w; v < primal_waves; v += nw)
            primal_wave<QM, LPI, UQ, EXP64>(g, t, count, LaneMap<LPI>(g.C, v));
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Many sweeps of a very small graph (every edge-chain and node-chain pair one
// thread of one work-group, q_max <= 5) with the state in LDS: x, the dual
// bits and the h records live in LDS and each thread keeps its edge's
// thresholds and its node's base in registers, so a sweep costs two barriers
// and no global memory round trip.  Draws and field sums are those of
// k_dual / k_primal (same generator calls, same compares, same FMA order),
// so the trajectory is bit-for-bit that of separate launches.  At the end x,
// the counters and the last sweep's dual words go back to global memory.
// LDS: h double [R][D] | counts u32 [n][QM] | pos u32 [n] | x u8 [n][C] |
// theta u8 [R][D][C], R = the nodes' segment entries in node order.
// ---------------------------------------------------------------------------
template <int QM, bool UQ, bool EXP64>
__global__ __launch_bounds__(1024) void k_sweeps_lds(Graph g, uint32_t t0, int32_t nsw,
                                                     int64_t burn_in, uint32_t R)
{
    static_assert(QM <= 5, "thresholds kept in registers");
    constexpr int D = dim_d(QM);
    extern __shared__ __align__(16) uint8_t sm[];
    const int n = (int)g.n, C = g.C, S = (int)g.hwm;
    double *hl = reinterpret_cast<double *>(sm);
    uint32_t *cl = reinterpret_cast<uint32_t *>(hl + (size_t)R * D);
    uint32_t *pos = cl + (size_t)n * QM;
    uint8_t *xl = reinterpret_cast<uint8_t *>(pos + n);
    uint8_t *tl = xl + (size_t)n * C;
    const int tid = threadIdx.x, nt = blockDim.x;
    if (tid == 0) {
        uint32_t a = 0;
        for (int i = 0; i < n; ++i) {
            pos[i] = a;
            a += g.inc_cnt[i];
        }
    }
    for (int k = tid; k < n * C; k += nt) xl[k] = g.x[k];
    for (int k = tid; k < n * QM; k += nt) cl[k] = 0u;
    for (int k = tid; k < (int)R * D * C; k += nt) tl[k] = 0;
    __syncthreads();
    for (int i = tid; i < n; i += nt) {
        const uint32_t o = g.inc_off[i], cn = g.inc_cnt[i], p0 = pos[i];
        for (uint32_t k = 0; k < cn; ++k)
            for (int dp = 0; dp < D; ++dp) hl[(size_t)(p0 + k) * D + dp] = g.rec_p[(uint64_t)(o + k) * D + dp];
    }
    // this thread's edge-chain item (dual) and node-chain item (primal)
    const bool de = tid < S * C;
    const int e = de ? tid / C : 0, ce = de ? tid % C : 0;
    const uint64_t uid = de ? g.uid[e] : 0ull;
    const bool dlive = uid != 0;
    int src = 0, dst = 0, qs = QM, qd = QM;
    uint32_t rs = 0, rd = 0;
    uint64_t sign = 0;
    uint32_t thr[2 * D];
#pragma unroll
    for (int d = 0; d < 2 * D; ++d) thr[d] = 0u;
    if (dlive) {
        src = g.src[e];
        dst = g.dst[e];
        if (!UQ) {
            qs = (int)(g.sq[e] & 15u);
            qd = (int)(g.sq[e] >> 4);
        }
    }
    __syncthreads();  // pos and the h records complete
    if (dlive) {
        rs = pos[src] + (g.ipos[2 * (uint64_t)e] - g.inc_off[src]);
        rd = pos[dst] + (g.ipos[2 * (uint64_t)e + 1] - g.inc_off[dst]);
        const uint8_t *blk = g.dparams + (int64_t)e * thr_bytes(QM);
        sign = *reinterpret_cast<const uint64_t *>(blk);
        const uint32_t *th = reinterpret_cast<const uint32_t *>(blk + off_thr(QM));
#pragma unroll
        for (int d = 0; d < 2 * D; ++d) thr[d] = th[d];
    }
    const bool dn = tid < n * C;
    const int i = dn ? tid / C : 0, cn_ = dn ? tid % C : 0;
    const int qn = dn ? (UQ ? QM : (int)g.q[i]) : QM;
    double base[QM];
#pragma unroll
    for (int a = 0; a < QM; ++a) base[a] = dn && (UQ || a < qn) ? g.base[(int64_t)i * QM + a] : 0.0;
    const uint32_t rp = dn ? pos[i] : 0u, rc = dn ? g.inc_cnt[i] : 0u;
    const int De = UQ ? D : (qs - 1) * (qd - 1);
    const int64_t quad = i >> 2;
    // The generator words of a sweep do not depend on the state, so the next
    // sweep's first dual call and its primal call are made while this sweep's
    // node draw runs (straight-line code: both chains interleave); every lane
    // computes them, and only the stores are predicated.
    auto dual_call = [&](uint32_t t, int k) {
        return philox4x32_10((uint32_t)uid, (uint32_t)(uid >> 32),
                             (kPhaseDual << 30) | (uint32_t)(16 * ce + k), t, g.rk);
    };
    auto primal_call = [&](uint32_t t) {
        return philox4x32_10((uint32_t)quad, (uint32_t)(quad >> 32),
                             (kPhasePrimal << 30) | (uint32_t)cn_, t, g.rk);
    };
    Words wd = dual_call(t0 + 1u, 0), wq = primal_call(t0 + 1u);
    for (int sw = 0; sw < nsw; ++sw) {
        const uint32_t t = t0 + 1u + (uint32_t)sw;
        {
            const int xs = xl[src * C + ce], xd = xl[dst * C + ce];
#pragma unroll
            for (int k = 0; k < (D + 4) / 5; ++k) {
                if (!UQ && 5 * k >= De) break;
                const Words w = k == 0 ? wd : dual_call(t, k);
                const uint32_t W[5] = {w.w0, w.w1, w.w2, w.w3,
                                       fifth_w(w)};
#pragma unroll
                for (int j = 0; j < 5; ++j) {
                    const int dd = 5 * k + j;
                    if (dd >= D) break;
                    const int qdv = UQ ? QM : (qd > 1 ? qd : 2);
                    const int a = dd / (qdv - 1) + 1, b = dd % (qdv - 1) + 1;
                    const bool yh = (xs == a) != (((sign >> dd) & 1ull) != 0);
                    const bool yb = xd == b;
                    // theta = cp | (ch & (yh | y')) | (cm & yh & y'), as in k_dual
                    const bool cp = W[j] > thr[2 * dd], cm = W[j] >= thr[2 * dd + 1];
                    const bool ch = W[j] >= 0x80000000u;
                    const uint8_t th = (uint8_t)(cp || (ch && (yh || yb)) || (cm && yh && yb));
                    if (dlive && (UQ || dd < De)) {
                        tl[((size_t)rs * D + (a - 1) * (QM - 1) + (b - 1)) * C + ce] = th;
                        tl[((size_t)rd * D + (b - 1) * (QM - 1) + (a - 1)) * C + ce] = th;
                    }
                }
            }
        }
        __syncthreads();
        {
            double L[QM];
#pragma unroll
            for (int a = 0; a < QM; ++a) L[a] = base[a];
            for (uint32_t k = 0; k < rc; ++k) {
                const double *h = hl + (size_t)(rp + k) * D;
                const uint8_t *z = tl + (size_t)(rp + k) * D * C + cn_;
#pragma unroll
                for (int s = 1; s < QM; ++s) {
                    if (!UQ && s >= qn) break;
                    double acc = L[s];
#pragma unroll
                    for (int o = 1; o < QM; ++o) {
                        const int dp = (s - 1) * (QM - 1) + (o - 1);
                        acc = __builtin_fma(__hiloint2double(z[dp * C] ? 0x40000000 : 0, 0), h[dp], acc);
                    }
                    L[s] = acc;
                }
            }
            const Words wd_next = dual_call(t + 1u, 0), wq_next = primal_call(t + 1u);
            const int xn = draw_node<QM, UQ, EXP64>(L, qn, word_at(wq, i & 3) >> 8);
            if (dn) {
                xl[i * C + cn_] = (uint8_t)xn;
                if ((int64_t)t > burn_in) atomicAdd(&cl[i * QM + xn], 1u);
            }
            wd = wd_next;
            wq = wq_next;
        }
        __syncthreads();
    }
    for (int k = tid; k < n * C; k += nt) g.x[k] = xl[k];
    for (int k = tid; k < n * QM; k += nt)
        if (cl[k]) g.counts[k] += cl[k];
    // the last sweep's dual words, in the records' global layout (entries
    // [0, used) of the compact order belong to segments)
    const uint32_t used = pos[n - 1] + g.inc_cnt[n - 1];
    for (int k = tid; k < (int)used * D; k += nt) {
        const uint32_t r = (uint32_t)(k / D);
        const int dp = k - (int)r * D;
        int lo = 0, hi = n - 1;  // node owning compact record r
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (pos[mid] <= r) lo = mid; else hi = mid - 1;
        }
        const uint64_t pr = (uint64_t)g.inc_off[lo] + (r - pos[lo]);
        uint32_t word = 0;
        for (int c = 0; c < C; ++c)
            if (tl[((size_t)r * D + dp) * C + c]) word |= 1u << c;
        g.rec_z[rec_zword(g, pr, dp, 0, D)] = word;
    }
}

// ---------------------------------------------------------------------------
// Small kernels: edits, readout.
// ---------------------------------------------------------------------------
// The device sweep counter of replayed sweeps: set before a replay, advanced
// by one at the start of each captured sweep.
__global__ void k_tick(uint32_t *t)
{
    if (threadIdx.x == 0) *t += 1u;
}
__global__ void k_set_counter(uint32_t *t, uint32_t v)
{
    if (threadIdx.x == 0) *t = v;
}

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

// theta of m edges (given by slot) for every chain: out [m][C], bit d for the
// edge's own entries d = (a-1)(q_dst-1) + (b-1), read from its src record.
__global__ void k_get_duals(int64_t m, int32_t QM, Graph g, const int32_t *__restrict__ slots,
                            uint64_t *__restrict__ out)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= m * g.C) return;
    const int64_t k = idx / g.C;
    const int c = (int)(idx - k * g.C);
    const int64_t s = slots[k];
    const uint32_t sq = g.sq[s];
    const int qs = (int)(sq & 15u), qd = (int)(sq >> 4);
    const uint64_t r0 = g.ipos[2 * s];
    uint64_t bits = 0;
    for (int d = 0; d < (qs - 1) * (qd - 1); ++d) {
        const int dp = (d / (qd - 1)) * (QM - 1) + d % (qd - 1);
        bits |= (uint64_t)rec_theta(g, r0, dp, c, QM) << d;
    }
    out[idx] = bits;
}

// New edges: copy h of the parameter block into both incidence records, each
// in its node's orientation (|h| on the dst side).  One thread per (edge,
// entry).
__global__ void k_write_records(int64_t m, int32_t QM, const int32_t *__restrict__ slots,
                                const uint8_t *__restrict__ sq, const uint8_t *__restrict__ params,
                                const uint32_t *__restrict__ ipos, double *__restrict__ rec_p)
{
    const int RP = rec_len(QM);
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= m * RP) return;
    const int64_t k = idx / RP;
    const int j = (int)(idx - k * RP);
    const int64_t s = slots[k];
    const uint8_t *blk = params + s * block_bytes(QM);
    const double *h = reinterpret_cast<const double *>(blk + off_h(QM));
    const int qs = (int)(sq[s] & 15u), qd = (int)(sq[s] >> 4);
    double vs = 0.0, vd = 0.0;
    // src record: row j / (QM-1) is the src state; dst record: the dst state
    const int r = j / (QM - 1) + 1, o = j % (QM - 1) + 1;
    if (r < qs && o < qd) vs = h[(r - 1) * (qd - 1) + (o - 1)];
    if (o < qs && r < qd) vd = fabs(h[(o - 1) * (qd - 1) + (r - 1)]);
    rec_p[(uint64_t)ipos[2 * s] * RP + j] = vs;
    rec_p[(uint64_t)ipos[2 * s + 1] * RP + j] = vd;
}

// base of the listed nodes (the first *count of them when count is given):
// lam plus the c0 of each live incidence (from the edge's parameter block,
// the node's side).  One wave per node: lane l sums
// records l, l + 64, ... and the wave adds the lanes' sums in a fixed butterfly,
// so the result depends only on the node's record list.
template <int QM>
__global__ __launch_bounds__(256) void k_node_base(int64_t nn, const uint32_t *__restrict__ count,
                                                   const uint32_t *__restrict__ nodes,
                                                   const double *__restrict__ lam,
                                                   const uint32_t *__restrict__ off,
                                                   const uint32_t *__restrict__ cnt,
                                                   const uint32_t *__restrict__ inc,
                                                   const uint8_t *__restrict__ params,
                                                   double *__restrict__ base)
{
    const int64_t k = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (k >= nn || (count && k >= (int64_t)*count)) return;
    const uint64_t i = nodes[k];
    double acc[QM];
#pragma unroll
    for (int a = 0; a < QM; ++a) acc[a] = 0.0;
    const uint32_t o = off[i], n = cnt[i];
    // a lane adds its records r = lane, lane + 64, ... in that order; four at
    // a time, with every load issued before any is used (entries past the end
    // re-read the last one, tombstones read block 0, and both add nothing),
    // so a hub's wave waits once per four records instead of once per record
    constexpr int U = 4;
    for (uint32_t r0 = lane; r0 < n; r0 += 64 * U) {
        uint32_t e[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t r = r0 + 64u * u;
            const uint32_t v = inc[o + (r < n ? r : n - 1u)];
            e[u] = r < n ? v : kTomb;
        }
        double c[U][QM - 1];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool live = e[u] != kTomb;
            const double *c0 = reinterpret_cast<const double *>(
                params + (live ? (int64_t)(e[u] >> 1) * block_bytes(QM) : 0) + off_c0(QM));
            const uint32_t side = live ? (e[u] & 1u) : 0u;
#pragma unroll
            for (int a = 1; a < QM; ++a) c[u][a - 1] = c0[side * (QM - 1) + (a - 1)];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (e[u] != kTomb)
#pragma unroll
                for (int a = 1; a < QM; ++a) acc[a] += c[u][a - 1];
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
#pragma unroll
        for (int a = 1; a < QM; ++a) acc[a] += __shfl_xor(acc[a], m);
    double v = 0.0;
#pragma unroll
    for (int a = 1; a < QM; ++a)
        if (lane == a) v = acc[a];
    if (lane < QM) base[i * QM + lane] = lam[i * QM + lane] + v;
}

// New edges: keep their log tables (row = src state) for the estimator below.
// Sign word and thresholds of the new edges' blocks into the dual's array
// (words: thr_bytes / 4 per slot; bb: block bytes).
__global__ void k_copy_dual_params(int64_t m, int32_t words, int64_t bb,
                                   const int32_t *__restrict__ slots,
                                   const uint8_t *__restrict__ params, uint8_t *__restrict__ dparams)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= m * words) return;
    const int64_t k = idx / words, w = idx - k * words, sl = slots[k];
    reinterpret_cast<uint32_t *>(dparams)[sl * words + w] =
        *reinterpret_cast<const uint32_t *>(params + sl * bb + 4 * w);
}

template <typename T>
__global__ void k_copy_tables(int64_t m, int32_t QQ, const int32_t *__restrict__ slots,
                              const T *__restrict__ phi, T *__restrict__ lphi)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= m * QQ) return;
    const int64_t k = idx / QQ;
    lphi[(int64_t)slots[k] * QQ + (idx - k * QQ)] = phi[idx];
}

// ---------------------------------------------------------------------------
// Sec. 5.2: the estimator V(x, theta) = p~(x) p~(theta) / p~(x, theta) of the
// partition function.  By the Lemma of Sec. 3, p~(theta) / p~(x, theta) =
// 1 / p(x | theta), which factorizes over the nodes, so per chain
//   log V = sum_i lam_i(x_i) + sum_e Lam_e(x_src, x_dst)
//           - sum_i [L_i(x_i) - log sum_a exp L_i(a)],
// L_i the node field given theta (the primal phase's).  Evaluated between
// the phases of a sweep, x being the state the duals were drawn from.  Lane =
// chain; a block of four waves covers 16 nodes (a quad per wave) or 64 edges
// (16 per wave) for one block of 64 chains and writes one row of partial sums
// part[row][CB][64]; k_logv_reduce adds the rows of a chain in a fixed order,
// so the value does not depend on scheduling.
// ---------------------------------------------------------------------------
constexpr int kLvEdges = 16;  // edges per wave

// Node part: lam_i(x_i) - log p(x_i | theta) over the block's 16 nodes.  Removed
// edges leave zero records, which add nothing, so records are not tested.
template <int QM, bool W64>
__global__ __launch_bounds__(256) void k_logv_nodes(Graph g, double *__restrict__ part)
{
    constexpr int D = dim_d(QM);
    constexpr int U = D <= 9 ? 2 : 1;  // records whose loads go out together
    constexpr int ZS = W64 ? 2 : 1;    // u32 mask words between entries (64-bit words with C > 32)
    __shared__ double red[4][64];
    const int wib = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int cb = blockIdx.y, c = cb * 64 + lane;
    const bool cv = c < g.C;
    const bool zc = zc_layout(QM, g.C);
    const int64_t quad = (int64_t)blockIdx.x * 4 + wib;
    // the quad's headers first
    uint32_t off[4], cnt[4];
    int xq[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t i = quad * 4 + j;
        const bool in = i < g.n;
        off[j] = in ? g.inc_off[i] : 0u;
        cnt[j] = in ? g.inc_cnt[i] : 0u;
        xq[j] = in && cv ? (int)g.x[i * g.C + c] : 0;
    }
    double acc = 0.0, zq = 1.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t i = quad * 4 + j;
        if (i >= g.n) break;
        const int qn = (int)g.q[i];
        double L[QM];
#pragma unroll
        for (int a = 0; a < QM; ++a) L[a] = g.base[i * QM + a];  // finite past q_i
        const uint32_t o = off[j], end = off[j] + cnt[j];
        for (uint32_t r = o; r < end; r += U) {
            // U records (clamped to the segment; extra ones add zero)
            double hv[U][D];
            uint32_t zw[U][D];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t rr = r + u < end ? r + u : end - 1;
                const double *h = g.rec_p + (uint64_t)rr * D;
                if (zc) {
                    // chain-major words: chain c's bit of entry dp moved to bit c
                    const uint64_t wz =
                        cv ? reinterpret_cast<const uint64_t *>(g.rec_z)[(uint64_t)rr * g.C + c] : 0ull;
#pragma unroll
                    for (int dp = 0; dp < D; ++dp) {
                        hv[u][dp] = h[dp];
                        zw[u][dp] = ((uint32_t)(wz >> (8 * (dp / (QM - 1)) + dp % (QM - 1))) & 1u)
                                    << (c & 31);
                    }
                } else {
                    const uint32_t *z = g.rec_z + rec_zword(g, rr, 0, c, D);
#pragma unroll
                    for (int dp = 0; dp < D; ++dp) {
                        hv[u][dp] = h[dp];
                        zw[u][dp] = z[dp * ZS];
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (r + u >= end) break;
#pragma unroll
                for (int s = 1; s < QM; ++s)
#pragma unroll
                    for (int oo = 1; oo < QM; ++oo) {
                        const int dp = (s - 1) * (QM - 1) + (oo - 1);
                        // + 2 theta h: factor 0.0 or 2.0, 2h exact
                        const double f = __hiloint2double(
                            ((zw[u][dp] >> (c & 31)) & 1u) ? 0x40000000 : 0, 0);
                        L[s] = __builtin_fma(f, hv[u][dp], L[s]);
                    }
            }
        }
        // log sum_a e^L(a) = mx + log z, z = 1 + sum over the other states of
        // e^(L(a) - mx) in [1, q_i]; the z of the quad's nodes are multiplied
        // and their log taken once
        const int xi = xq[j];
        double mx = L[0], lx = L[0];
        int am = 0;
#pragma unroll
        for (int a = 1; a < QM; ++a) {
            if (a < qn && L[a] > mx) {
                mx = L[a];
                am = a;
            }
            if (a == xi) lx = L[a];
        }
        double z = 1.0;
#pragma unroll
        for (int a = 0; a < QM; ++a)
            if (a < qn && a != am) z += exp(L[a] - mx);
        zq *= z;
        acc += g.lam[i * QM + xi] - (lx - mx);
    }
    acc += log(zq);
    red[wib][lane] = cv ? acc : 0.0;
    __syncthreads();
    if (wib == 0)
        part[((int64_t)blockIdx.x * g.CB + cb) * 64 + lane] =
            (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

// Edge part: Lam_e(x_src, x_dst) over the block's 64 slots (free slots skipped),
// from the log tables kept at insert.  A wave issues the loads of its 16
// edges together.
template <int QM, typename T>
__global__ __launch_bounds__(256) void k_logv_edges(Graph g, const T *__restrict__ lphi,
                                                    double *__restrict__ part)
{
    __shared__ double red[4][64];
    const int wib = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int cb = blockIdx.y, c = cb * 64 + lane;
    const bool cv = c < g.C;
    const int64_t e0 = ((int64_t)blockIdx.x * 4 + wib) * kLvEdges;
    double acc = 0.0;
    if (cv) {
        int32_t sa[kLvEdges], da[kLvEdges];
        bool live[kLvEdges];
#pragma unroll
        for (int k = 0; k < kLvEdges; ++k) {
            const int64_t e = e0 + k;
            live[k] = e < g.hwm && g.uid[e] != 0;
            sa[k] = live[k] ? g.src[e] : 0;
            da[k] = live[k] ? g.dst[e] : 0;
        }
        int xa[kLvEdges], xb[kLvEdges];
#pragma unroll
        for (int k = 0; k < kLvEdges; ++k) {
            xa[k] = g.x[(int64_t)sa[k] * g.C + c];
            xb[k] = g.x[(int64_t)da[k] * g.C + c];
        }
#pragma unroll
        for (int k = 0; k < kLvEdges; ++k)
            if (live[k]) acc += (double)lphi[((e0 + k) * QM + xa[k]) * QM + xb[k]];
    }
    red[wib][lane] = acc;
    __syncthreads();
    if (wib == 0)
        part[((int64_t)blockIdx.x * g.CB + cb) * 64 + lane] =
            (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

// Rows [b chunk, (b + 1) chunk) of part[rows][CB][64] summed per chain into
// out[b][CB][64] (block (b, cb), 64 threads; eight accumulators, fixed order).
__global__ __launch_bounds__(64) void k_logv_reduce(int64_t rows, int64_t chunk, int32_t CB,
                                                    const double *__restrict__ part,
                                                    double *__restrict__ out)
{
    const int64_t b = blockIdx.x;
    const int cb = blockIdx.y, l = threadIdx.x;
    const int64_t k0 = b * chunk, k1 = k0 + chunk < rows ? k0 + chunk : rows;
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t k = k0;
    for (; k + 8 <= k1; k += 8)
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] += part[((k + u) * CB + cb) * 64 + l];
    for (; k < k1; ++k) a[0] += part[(k * CB + cb) * 64 + l];
    out[(b * CB + cb) * 64 + l] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// pdg_set_state's check: flag any x[i][c] >= q_i.
__global__ void k_check_state(int64_t n, int C, const uint8_t *__restrict__ q,
                              const uint8_t *__restrict__ x, uint32_t *__restrict__ flag)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n * C && x[i] >= q[i / C]) *flag = 1u;
}

__global__ void k_marginals(int64_t nq, const uint32_t *__restrict__ counts, double samples,
                            double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nq) out[i] = samples > 0.0 ? (double)counts[i] / samples : 0.0;
}

}  // namespace pdg

// libpdg: host runtime and C ABI of the primal-dual Gibbs sweep (include/pdg.h).
//
// The context owns every device buffer.  Sweeps are two kernels per sweep on
// the caller's stream.  Edge edits are decided on the host -- a slot
// allocator (free stack, generation-tagged uids) and per-node incidence
// segments with slack -- and written to the device by small scatter kernels,
// so an edit batch costs O(batch) plus an occasional segment relocation; no
// colouring and no rebuild of the incidence lists is ever needed (the
// abstract, Sec. 1 and Sec. 6 of the paper motivate the method by exactly
// this setting).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "pdg.h"
#include "pdg_kernels.hpp"

namespace pdg {

static thread_local std::string g_global_err;

// Host mirror of the edge store, laid out so that an edit touches one cache
// line per slot and one per node.
struct SlotRec {
    uint64_t uid;        // 0 = free
    int32_t src, dst;
    uint32_t pos0, pos1; // position of the slot's entry in its src / dst segment
    uint32_t gen;        // generation of the slot (high word of its uids)
    uint32_t pad;
};
struct NodeRec {
    uint32_t off, cnt, cap, nlive;  // segment [off, off + cnt) of cap entries, live ones
};
struct Store {
    int64_t S = 0;
    std::vector<SlotRec> slot;    // [S]
    std::vector<int32_t> free_stack;
    int64_t hwm = 0, live = 0;
    std::vector<NodeRec> node;    // [n]
    std::vector<uint32_t> mark;                  // per node, zero between calls (edit scratch)
    std::vector<uint32_t> pool;
    int64_t pool_top = 0;
};

}  // namespace pdg

struct pdg_ctx {
    pdg_config cfg{};
    int device = 0;
    hipStream_t stream = nullptr;
    int QM = 0, D = 0, C = 0, LPI = 0, CB = 0;
    int RP = 0;       // doubles per incidence record
    int64_t ZW = 0;   // u32 mask words per incidence record
    int64_t bbytes = 0;
    int64_t n = 0;
    bool nodes_set = false;
    bool uq = false;  // every node has q_max states
    int64_t t = 0;
    int phase = 0;  // 0: between sweeps, 1: dual done
    int64_t counted = 0;
    // device
    uint8_t *d_q = nullptr;
    double *d_lam = nullptr;
    uint8_t *d_x = nullptr;
    uint32_t *d_counts = nullptr;
    double *d_base = nullptr;  // [n][QM] lam + c0 of the node's incidences
    int32_t *d_src = nullptr, *d_dst = nullptr;
    uint64_t *d_uid = nullptr;
    uint8_t *d_sq = nullptr;
    uint8_t *d_params = nullptr;
    uint32_t *d_ipos = nullptr;
    uint32_t *d_off = nullptr, *d_cnt = nullptr;
    uint32_t *d_pool = nullptr;
    double *d_rec_p = nullptr;
    uint32_t *d_rec_z = nullptr;
    int64_t dev_pool_cap = 0;
    uint32_t *d_flag = nullptr;
    void *d_scratch = nullptr;
    int64_t scratch_bytes = 0;
    // hubs (nodes with more than kHubThreshold incidence entries): their list,
    // piece table and partial fields
    uint32_t hub_thr = 0;        // threshold in force (0: hubs are not split)
    int64_t nh = 0, np = 0;      // hubs, pieces
    uint32_t *d_hub = nullptr;   // hnode[nh] | hpfirst[nh + 1] | pnode[np] | pfirst[np] | pn[np]
    int64_t hub_cap = 0;         // u32 capacity of d_hub
    double *d_part = nullptr;    // [np][CB][QM - 1][64]
    int64_t part_cap = 0;        // doubles
    pdg::Store st;
    std::string err;
};

namespace pdg {

static pdg_status fail(pdg_ctx *ctx, pdg_status code, const std::string &msg)
{
    if (ctx)
        ctx->err = msg;
    else
        g_global_err = msg;
    return code;
}

#define PDG_HIP(ctx, expr)                                                                  \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((ctx), PDG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define PDG_TRY(expr)                  \
    do {                               \
        pdg_status s_ = (expr);        \
        if (s_ != PDG_OK) return s_;   \
    } while (0)

static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
static inline unsigned grid_for(int64_t threads, int block = 256)
{
    return (unsigned)cdiv(std::max<int64_t>(threads, 1), block);
}

static int choose_lpi(int C)
{
    if (C >= 33) return 64;
    if (C >= 17) return 32;
    if (C >= 9) return 16;
    if (C >= 2) return 8;
    return 1;
}

static pdg_status dalloc(pdg_ctx *ctx, void **p, int64_t bytes)
{
    *p = nullptr;
    if (bytes <= 0) return PDG_OK;
    hipError_t e = hipMalloc(p, (size_t)bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(ctx, PDG_ENOMEM,
                    "hipMalloc(" + std::to_string(bytes) + "): " + hipGetErrorString(e));
    }
    return PDG_OK;
}

static pdg_status scratch(pdg_ctx *ctx, int64_t bytes, void **out)
{
    if (bytes > ctx->scratch_bytes) {
        if (ctx->d_scratch) PDG_HIP(ctx, hipFree(ctx->d_scratch));
        ctx->d_scratch = nullptr;
        ctx->scratch_bytes = 0;
        int64_t want = std::max<int64_t>(bytes, 1 << 20);
        PDG_TRY(dalloc(ctx, &ctx->d_scratch, want));
        ctx->scratch_bytes = want;
    }
    *out = ctx->d_scratch;
    return PDG_OK;
}

static pdg_status set_dev(pdg_ctx *ctx)
{
    PDG_HIP(ctx, hipSetDevice(ctx->device));
    return PDG_OK;
}

static pdg_status read_flag(pdg_ctx *ctx, uint32_t *h)
{
    PDG_HIP(ctx, hipMemcpyAsync(h, ctx->d_flag, 4, hipMemcpyDeviceToHost, ctx->stream));
    PDG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return PDG_OK;
}

static pdg_status clear_flag(pdg_ctx *ctx)
{
    k_fill_u32<<<1, 64, 0, ctx->stream>>>(ctx->d_flag, 1, 0u);
    PDG_HIP(ctx, hipGetLastError());
    return PDG_OK;
}

static Graph make_graph(pdg_ctx *ctx)
{
    Graph g;
    g.q = ctx->d_q;
    g.lam = ctx->d_lam;
    g.src = ctx->d_src;
    g.dst = ctx->d_dst;
    g.uid = ctx->d_uid;
    g.sq = ctx->d_sq;
    g.params = ctx->d_params;
    g.ipos = ctx->d_ipos;
    g.base = ctx->d_base;
    g.inc_off = ctx->d_off;
    g.inc_cnt = ctx->d_cnt;
    g.inc = ctx->d_pool;
    g.rec_p = ctx->d_rec_p;
    g.rec_z = ctx->d_rec_z;
    g.x = ctx->d_x;
    g.counts = ctx->d_counts;
    g.n = ctx->n;
    g.hwm = ctx->st.hwm;
    g.C = ctx->C;
    g.CB = (int32_t)cdiv(ctx->C, 64);
    g.heavy = ctx->hub_thr;
    g.k0 = (uint32_t)ctx->cfg.seed;
    g.k1 = (uint32_t)(ctx->cfg.seed >> 32);
    g.rk = make_round_keys(ctx->cfg.seed);
    return g;
}

// ------------------------------------------------------------- kernel dispatch
template <int QM, int LPI, bool UQ>
static void launch_dual_t(const Graph &g, uint32_t t, int CB, hipStream_t s)
{
    if constexpr (LPI == 64) {
        constexpr int E = kDualEdgesPerWave;
        const int64_t waves = cdiv(g.hwm, E) * CB;
        k_dual64<QM, UQ, E><<<grid_for(waves * 64), 256, 0, s>>>(g, t);
    } else {
        constexpr int P = 64 / LPI;
        const int64_t waves = cdiv(g.hwm, P) * CB;
        k_dual<QM, LPI, UQ><<<grid_for(waves * 64), 256, 0, s>>>(g, t);
    }
}

template <int QM, int LPI, bool UQ, bool E64>
static void launch_primal_t(const Graph &g, uint32_t t, int count, int CB, hipStream_t s)
{
    constexpr int P = 64 / LPI;
    if constexpr (LPI == 64) {
        const int64_t waves = cdiv(g.n, 4) * CB;
        k_primal64<QM, UQ, E64><<<grid_for(waves * 64), 256, 0, s>>>(g, t, count);
    } else if constexpr (LPI == 32) {
        const int64_t waves = cdiv(g.n, 4);  // one quad per wave, halves split the records
        k_primal32<QM, UQ, E64><<<grid_for(waves * 64), 256, 0, s>>>(g, t, count);
    } else {
        const int64_t waves = cdiv(cdiv(g.n, 4), P) * CB;
        k_primal<QM, LPI, UQ, E64><<<grid_for(waves * 64), 256, 0, s>>>(g, t, count);
    }
}

template <int QM, bool UQ>
static void dual_q(int lpi, const Graph &g, uint32_t t, int CB, hipStream_t s)
{
    switch (lpi) {
    case 1: launch_dual_t<QM, 1, UQ>(g, t, CB, s); break;
    case 8: launch_dual_t<QM, 8, UQ>(g, t, CB, s); break;
    case 16: launch_dual_t<QM, 16, UQ>(g, t, CB, s); break;
    case 32: launch_dual_t<QM, 32, UQ>(g, t, CB, s); break;
    default: launch_dual_t<QM, 64, UQ>(g, t, CB, s); break;
    }
}

template <int QM, bool UQ, bool E64>
static void primal_q(int lpi, const Graph &g, uint32_t t, int count, int CB, hipStream_t s)
{
    switch (lpi) {
    case 1: launch_primal_t<QM, 1, UQ, E64>(g, t, count, CB, s); break;
    case 8: launch_primal_t<QM, 8, UQ, E64>(g, t, count, CB, s); break;
    case 16: launch_primal_t<QM, 16, UQ, E64>(g, t, count, CB, s); break;
    case 32: launch_primal_t<QM, 32, UQ, E64>(g, t, count, CB, s); break;
    default: launch_primal_t<QM, 64, UQ, E64>(g, t, count, CB, s); break;
    }
}

template <bool UQ>
static void launch_dual_u(pdg_ctx *ctx, uint32_t t)
{
    const Graph g = make_graph(ctx);
    switch (ctx->QM) {
    case 2: dual_q<2, UQ>(ctx->LPI, g, t, ctx->CB, ctx->stream); break;
    case 3: dual_q<3, UQ>(ctx->LPI, g, t, ctx->CB, ctx->stream); break;
    case 4: dual_q<4, UQ>(ctx->LPI, g, t, ctx->CB, ctx->stream); break;
    case 5: dual_q<5, UQ>(ctx->LPI, g, t, ctx->CB, ctx->stream); break;
    case 6: dual_q<6, UQ>(ctx->LPI, g, t, ctx->CB, ctx->stream); break;
    case 7: dual_q<7, UQ>(ctx->LPI, g, t, ctx->CB, ctx->stream); break;
    default: dual_q<8, UQ>(ctx->LPI, g, t, ctx->CB, ctx->stream); break;
    }
}

static void launch_dual(pdg_ctx *ctx, uint32_t t)
{
    if (ctx->uq)
        launch_dual_u<true>(ctx, t);
    else
        launch_dual_u<false>(ctx, t);
}

template <int QM, bool UQ, bool E64>
static void launch_hubs_q(pdg_ctx *ctx, const Graph &g, uint32_t t, int count)
{
    const uint32_t *hn = ctx->d_hub, *hp = hn + ctx->nh, *pnode = hp + ctx->nh + 1;
    const uint32_t *pf = pnode + ctx->np, *pn = pf + ctx->np;
    const int64_t wp = ctx->np * ctx->CB, wf = ctx->nh * ctx->CB;
    if (ctx->LPI == 64) {
        k_hub_pieces<QM, 64><<<grid_for(wp * 64), 256, 0, ctx->stream>>>(g, ctx->np, pnode, pf, pn,
                                                                         ctx->d_part);
        k_hub_finish<QM, UQ, E64, 64><<<grid_for(wf * 64), 256, 0, ctx->stream>>>(
            g, ctx->nh, hn, hp, ctx->d_part, t, count);
    } else {
        k_hub_pieces<QM, 32><<<grid_for(wp * 64), 256, 0, ctx->stream>>>(g, ctx->np, pnode, pf, pn,
                                                                         ctx->d_part);
        k_hub_finish<QM, UQ, E64, 32><<<grid_for(wf * 64), 256, 0, ctx->stream>>>(
            g, ctx->nh, hn, hp, ctx->d_part, t, count);
    }
}

template <bool UQ, bool E64>
static void launch_primal_e(pdg_ctx *ctx, uint32_t t, int count)
{
    const Graph g = make_graph(ctx);
    switch (ctx->QM) {
    case 2: primal_q<2, UQ, E64>(ctx->LPI, g, t, count, ctx->CB, ctx->stream); break;
    case 3: primal_q<3, UQ, E64>(ctx->LPI, g, t, count, ctx->CB, ctx->stream); break;
    case 4: primal_q<4, UQ, E64>(ctx->LPI, g, t, count, ctx->CB, ctx->stream); break;
    case 5: primal_q<5, UQ, E64>(ctx->LPI, g, t, count, ctx->CB, ctx->stream); break;
    case 6: primal_q<6, UQ, E64>(ctx->LPI, g, t, count, ctx->CB, ctx->stream); break;
    case 7: primal_q<7, UQ, E64>(ctx->LPI, g, t, count, ctx->CB, ctx->stream); break;
    default: primal_q<8, UQ, E64>(ctx->LPI, g, t, count, ctx->CB, ctx->stream); break;
    }
    if (g.heavy && ctx->nh) {
        switch (ctx->QM) {
        case 2: launch_hubs_q<2, UQ, E64>(ctx, g, t, count); break;
        case 3: launch_hubs_q<3, UQ, E64>(ctx, g, t, count); break;
        case 4: launch_hubs_q<4, UQ, E64>(ctx, g, t, count); break;
        case 5: launch_hubs_q<5, UQ, E64>(ctx, g, t, count); break;
        case 6: launch_hubs_q<6, UQ, E64>(ctx, g, t, count); break;
        case 7: launch_hubs_q<7, UQ, E64>(ctx, g, t, count); break;
        default: launch_hubs_q<8, UQ, E64>(ctx, g, t, count); break;
        }
    }
}

static void launch_primal(pdg_ctx *ctx, uint32_t t, int count)
{
    const bool e64 = ctx->cfg.precision == PDG_PRECISION_F64;
    if (ctx->uq) {
        if (e64) launch_primal_e<true, true>(ctx, t, count);
        else launch_primal_e<true, false>(ctx, t, count);
    } else {
        if (e64) launch_primal_e<false, true>(ctx, t, count);
        else launch_primal_e<false, false>(ctx, t, count);
    }
}

template <int QM>
static void decompose_q(bool f64, int64_t m, const int32_t *qs, const int32_t *qd, const void *phi,
                        const int32_t *dest, uint8_t *out, uint32_t *bad, hipStream_t s)
{
    if (f64)
        k_decompose<QM, double><<<grid_for(m, 128), 128, 0, s>>>(
            m, qs, qd, static_cast<const double *>(phi), dest, out, bad);
    else
        k_decompose<QM, float><<<grid_for(m, 128), 128, 0, s>>>(
            m, qs, qd, static_cast<const float *>(phi), dest, out, bad);
}

static void launch_decompose(int qm, bool f64, int64_t m, const int32_t *qs, const int32_t *qd,
                             const void *phi, const int32_t *dest, uint8_t *out, uint32_t *bad,
                             hipStream_t s)
{
    switch (qm) {
    case 2: decompose_q<2>(f64, m, qs, qd, phi, dest, out, bad, s); break;
    case 3: decompose_q<3>(f64, m, qs, qd, phi, dest, out, bad, s); break;
    case 4: decompose_q<4>(f64, m, qs, qd, phi, dest, out, bad, s); break;
    case 5: decompose_q<5>(f64, m, qs, qd, phi, dest, out, bad, s); break;
    case 6: decompose_q<6>(f64, m, qs, qd, phi, dest, out, bad, s); break;
    case 7: decompose_q<7>(f64, m, qs, qd, phi, dest, out, bad, s); break;
    default: decompose_q<8>(f64, m, qs, qd, phi, dest, out, bad, s); break;
    }
}

// Finite-entry check of an edit batch before anything is changed.
template <int QM, typename T>
__global__ void k_check_tables(int64_t m, const int32_t *__restrict__ src,
                               const int32_t *__restrict__ dst, const uint8_t *__restrict__ q,
                               const T *__restrict__ phi, uint32_t *__restrict__ bad)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const int qs = q[src[k]], qd = q[dst[k]];
    const T *L = phi + k * QM * QM;
    for (int a = 0; a < qs; ++a)
        for (int b = 0; b < qd; ++b)
            if (!isfinite((double)L[a * QM + b])) atomicOr(bad, 1u);
}

template <int QM>
static void check_q(bool f64, int64_t m, const int32_t *s, const int32_t *d, const uint8_t *q,
                    const void *phi, uint32_t *bad, hipStream_t st)
{
    if (f64)
        k_check_tables<QM, double><<<grid_for(m), 256, 0, st>>>(m, s, d, q,
                                                               static_cast<const double *>(phi), bad);
    else
        k_check_tables<QM, float><<<grid_for(m), 256, 0, st>>>(m, s, d, q,
                                                              static_cast<const float *>(phi), bad);
}

static void launch_check(int qm, bool f64, int64_t m, const int32_t *s, const int32_t *d,
                         const uint8_t *q, const void *phi, uint32_t *bad, hipStream_t st)
{
    switch (qm) {
    case 2: check_q<2>(f64, m, s, d, q, phi, bad, st); break;
    case 3: check_q<3>(f64, m, s, d, q, phi, bad, st); break;
    case 4: check_q<4>(f64, m, s, d, q, phi, bad, st); break;
    case 5: check_q<5>(f64, m, s, d, q, phi, bad, st); break;
    case 6: check_q<6>(f64, m, s, d, q, phi, bad, st); break;
    case 7: check_q<7>(f64, m, s, d, q, phi, bad, st); break;
    default: check_q<8>(f64, m, s, d, q, phi, bad, st); break;
    }
}

// ---------------------------------------------------------------- edge store
static uint32_t slack_for(uint32_t k) { return std::max<uint32_t>(2u, k / 4u); }

// Edits touch the host mirror at random places; the loops below request the
// lines of later iterations ahead of time (distance kAhead).
constexpr int64_t kAhead = 16;
template <typename T>
static inline void prefetch_w(const T *p)
{
    __builtin_prefetch(p, 1, 0);
}

struct Patches {
    std::vector<uint32_t> idx, val;        // pool entries
    bool full = false;                     // whole pool and every header re-laid
    std::vector<uint32_t> mv_from, mv_to;  // incidence records that moved
    std::vector<uint32_t> ip_key, ip_val;  // ipos[2 slot + side] = record index
};

static void note_entry(Store &st, uint32_t e, uint32_t w, uint32_t rec, Patches &P)
{
    const uint32_t slot = e >> 1;
    if (e & 1u)
        st.slot[slot].pos1 = w;
    else
        st.slot[slot].pos0 = w;
    P.ip_key.push_back(2u * slot + (e & 1u));
    P.ip_val.push_back(rec);
}

// Lay every node's live entries out again, leaving room for `need` appends.
static pdg_status full_compact(pdg_ctx *ctx, const std::vector<uint32_t> &need, Patches &P)
{
    Store &st = ctx->st;
    const int64_t n = ctx->n;
    std::vector<uint32_t> noff(n), ncap(n);
    uint64_t total = 0;
    for (int64_t i = 0; i < n; ++i) {
        const uint32_t want = st.node[i].nlive + need[i];
        ncap[i] = want ? want + slack_for(want) : 0;
        noff[i] = (uint32_t)total;
        total += ncap[i];
    }
    const uint64_t size = total + total / 4 + 1024;
    if (size >= 0xFFFFFFF0ull) return fail(ctx, PDG_ECAPACITY, "incidence pool exceeds 2^32 entries");
    std::vector<uint32_t> npool((size_t)size, kTomb);
    P.full = true;
    P.idx.clear();
    P.val.clear();
    P.mv_from.clear();
    P.mv_to.clear();
    for (int64_t i = 0; i < n; ++i) {
        uint32_t w = 0;
        for (uint32_t k = 0; k < st.node[i].cnt; ++k) {
            const uint32_t e = st.pool[st.node[i].off + k];
            if (e == kTomb) continue;
            npool[noff[i] + w] = e;
            P.mv_from.push_back(st.node[i].off + k);
            P.mv_to.push_back(noff[i] + w);
            note_entry(st, e, w, noff[i] + w, P);
            ++w;
        }
        st.node[i].off = noff[i];
        st.node[i].cnt = w;
        st.node[i].cap = ncap[i];
    }
    st.pool.swap(npool);
    st.pool_top = (int64_t)total;
    return PDG_OK;
}

static void relocate(pdg_ctx *ctx, int64_t i, uint32_t need, Patches &P)
{
    Store &st = ctx->st;
    const uint32_t want = st.node[i].nlive + need;
    const uint32_t ncap = want + slack_for(want);
    const uint32_t noff = (uint32_t)st.pool_top;
    st.pool_top += ncap;
    uint32_t w = 0;
    for (uint32_t k = 0; k < st.node[i].cnt; ++k) {
        const uint32_t e = st.pool[st.node[i].off + k];
        if (e == kTomb) continue;
        st.pool[noff + w] = e;
        P.idx.push_back(noff + w);
        P.val.push_back(e);
        P.mv_from.push_back(st.node[i].off + k);
        P.mv_to.push_back(noff + w);
        note_entry(st, e, w, noff + w, P);
        ++w;
    }
    st.node[i].off = noff;
    st.node[i].cnt = w;
    st.node[i].cap = ncap;
}

static void append(pdg_ctx *ctx, int64_t i, uint32_t e, Patches &P)
{
    Store &st = ctx->st;
    const uint32_t p = st.node[i].cnt++;
    st.pool[st.node[i].off + p] = e;
    if (!P.full) {
        P.idx.push_back(st.node[i].off + p);
        P.val.push_back(e);
    }
    note_entry(st, e, p, st.node[i].off + p, P);
    st.node[i].nlive++;
}

// Upload a host vector to a fresh region of the scratch buffer.
template <typename T>
static T *stage(pdg_ctx *ctx, char *&cursor, const std::vector<T> &v)
{
    T *p = reinterpret_cast<T *>(cursor);
    if (!v.empty())
        (void)hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, ctx->stream);
    cursor += ((v.size() * sizeof(T) + 255) / 256) * 256;
    return p;
}

// Push host-side changes of the incidence structure and its records to the
// device: record moves (into new buffers after a full re-layout), pool
// entries, segment headers and ipos.
static pdg_status upload(pdg_ctx *ctx, Patches &P, const std::vector<int64_t> &touched)
{
    Store &st = ctx->st;
    const int64_t nmv = (int64_t)P.mv_from.size();
    const int64_t np = (int64_t)P.idx.size();
    const int64_t nn = (int64_t)touched.size();
    const int64_t nip = (int64_t)P.ip_key.size();
    std::vector<uint32_t> hn(nn), ho(nn), hc(nn);
    for (int64_t k = 0; k < nn; ++k) {
        hn[k] = (uint32_t)touched[k];
        ho[k] = st.node[touched[k]].off;
        hc[k] = st.node[touched[k]].cnt;
    }
    void *s;
    PDG_TRY(scratch(ctx, 4 * (2 * nmv + 2 * np + 3 * nn + 2 * nip) + 8 * 256, &s));
    char *cur = static_cast<char *>(s);
    uint32_t *dmf = stage(ctx, cur, P.mv_from), *dmt = stage(ctx, cur, P.mv_to);
    uint32_t *di = stage(ctx, cur, P.idx), *dv = stage(ctx, cur, P.val);
    uint32_t *dn = stage(ctx, cur, hn), *dof = stage(ctx, cur, ho), *dc = stage(ctx, cur, hc);
    uint32_t *dk = stage(ctx, cur, P.ip_key), *dkv = stage(ctx, cur, P.ip_val);
    PDG_HIP(ctx, hipGetLastError());
    if (P.full) {
        // new pool, records moved into fresh buffers
        const int64_t cap = (int64_t)st.pool.size();
        uint32_t *npool = nullptr;
        double *nrp = nullptr;
        uint32_t *nrz = nullptr;
        PDG_TRY(dalloc(ctx, (void **)&npool, cap * 4));
        // the primal stages records in 16-byte pieces: pad past the last one
        pdg_status a = dalloc(ctx, (void **)&nrp, cap * ctx->RP * 8 + 256);
        if (a == PDG_OK) a = dalloc(ctx, (void **)&nrz, cap * ctx->ZW * 4 + 256);
        if (a != PDG_OK) {
            (void)hipFree(npool);
            if (nrp) (void)hipFree(nrp);
            return a;
        }
        PDG_HIP(ctx, hipMemsetAsync(nrp, 0, cap * ctx->RP * 8 + 256, ctx->stream));
        PDG_HIP(ctx, hipMemsetAsync(nrz, 0, cap * ctx->ZW * 4 + 256, ctx->stream));
        if (nmv && ctx->d_rec_p) {
            k_move_rec_p<<<grid_for(nmv * ctx->RP), 256, 0, ctx->stream>>>(nmv, ctx->RP, dmf, dmt,
                                                                          ctx->d_rec_p, nrp);
            k_move_rec_z<<<grid_for(nmv * ctx->ZW), 256, 0, ctx->stream>>>(nmv, ctx->ZW, dmf, dmt,
                                                                          ctx->d_rec_z, nrz);
            PDG_HIP(ctx, hipGetLastError());
        }
        PDG_HIP(ctx, hipMemcpyAsync(npool, st.pool.data(), cap * 4, hipMemcpyHostToDevice,
                                    ctx->stream));
        std::vector<uint32_t> all_off((size_t)ctx->n), all_cnt((size_t)ctx->n);
        for (int64_t i = 0; i < ctx->n; ++i) {
            all_off[i] = st.node[i].off;
            all_cnt[i] = st.node[i].cnt;
        }
        PDG_HIP(ctx, hipMemcpyAsync(ctx->d_off, all_off.data(), (size_t)ctx->n * 4,
                                    hipMemcpyHostToDevice, ctx->stream));
        PDG_HIP(ctx, hipMemcpyAsync(ctx->d_cnt, all_cnt.data(), (size_t)ctx->n * 4,
                                    hipMemcpyHostToDevice, ctx->stream));
        PDG_HIP(ctx, hipStreamSynchronize(ctx->stream));
        if (ctx->d_pool) PDG_HIP(ctx, hipFree(ctx->d_pool));
        if (ctx->d_rec_p) PDG_HIP(ctx, hipFree(ctx->d_rec_p));
        if (ctx->d_rec_z) PDG_HIP(ctx, hipFree(ctx->d_rec_z));
        ctx->d_pool = npool;
        ctx->d_rec_p = nrp;
        ctx->d_rec_z = nrz;
        ctx->dev_pool_cap = cap;
    } else {
        if (st.pool_top > ctx->dev_pool_cap)
            return fail(ctx, PDG_EINVAL, "internal: pool beyond device capacity without re-layout");
        if (nmv) {  // relocated segments land in unused pool space: no overlap
            k_move_rec_p<<<grid_for(nmv * ctx->RP), 256, 0, ctx->stream>>>(
                nmv, ctx->RP, dmf, dmt, ctx->d_rec_p, ctx->d_rec_p);
            k_move_rec_z<<<grid_for(nmv * ctx->ZW), 256, 0, ctx->stream>>>(
                nmv, ctx->ZW, dmf, dmt, ctx->d_rec_z, ctx->d_rec_z);
        }
        if (np) k_scatter_u32<<<grid_for(np), 256, 0, ctx->stream>>>(np, di, dv, ctx->d_pool);
        if (nn)
            k_scatter_nodes<<<grid_for(nn), 256, 0, ctx->stream>>>(nn, dn, dof, dc, ctx->d_off,
                                                                   ctx->d_cnt);
        PDG_HIP(ctx, hipGetLastError());
    }
    if (nip) {
        k_set_ipos<<<grid_for(nip), 256, 0, ctx->stream>>>(nip, dk, dkv, ctx->d_ipos);
        PDG_HIP(ctx, hipGetLastError());
    }
    PDG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return PDG_OK;
}

template <int QM>
static void node_base_q(pdg_ctx *ctx, int64_t nn, const uint32_t *dnodes)
{
    k_node_base<QM><<<grid_for(nn * 64), 256, 0, ctx->stream>>>(
        nn, dnodes, ctx->d_lam, ctx->d_off, ctx->d_cnt, ctx->d_pool, ctx->d_params, ctx->d_base);
}

// base of the listed nodes (after their incidence lists changed)
static void launch_node_base(pdg_ctx *ctx, int64_t nn, const uint32_t *dnodes)
{
    if (nn == 0) return;
    switch (ctx->QM) {
    case 2: node_base_q<2>(ctx, nn, dnodes); break;
    case 3: node_base_q<3>(ctx, nn, dnodes); break;
    case 4: node_base_q<4>(ctx, nn, dnodes); break;
    case 5: node_base_q<5>(ctx, nn, dnodes); break;
    case 6: node_base_q<6>(ctx, nn, dnodes); break;
    case 7: node_base_q<7>(ctx, nn, dnodes); break;
    default: node_base_q<8>(ctx, nn, dnodes); break;
    }
}

// Hub list and piece table from the host's segment counts (the device holds
// the same counts).  Hubs are split only with 32 or more chains and while a
// hub piece kernel's LDS chunk holds at least the records of one step.
static pdg_status rebuild_hubs(pdg_ctx *ctx)
{
    Store &st = ctx->st;
    ctx->hub_thr = 0;
    ctx->nh = ctx->np = 0;
    if (ctx->LPI < 32) return PDG_OK;
    const int64_t D = ctx->D, RP = ctx->RP;
    const int64_t zr = ctx->LPI == 64 ? 2 * D * ctx->CB : D;
    const int64_t zb = (8 * D + 15) / 16 * 16;
    const int64_t K = (4096 - zb - 48) / (RP * 8 + 4 * zr);
    if (K < (ctx->LPI == 32 ? 2 : 1)) return PDG_OK;
    std::vector<uint32_t> hn, hp{0}, pn_node, pf, pn;
    for (int64_t i = 0; i < ctx->n; ++i) {
        const uint32_t c = st.node[i].cnt;
        if (c <= kHubThreshold) continue;
        hn.push_back((uint32_t)i);
        for (uint32_t f = 0; f < c; f += kHubPiece) {
            pn_node.push_back((uint32_t)i);
            pf.push_back(f);
            pn.push_back(std::min(kHubPiece, c - f));
        }
        hp.push_back((uint32_t)pf.size());
    }
    const int64_t nh = (int64_t)hn.size(), np = (int64_t)pf.size();
    if (nh == 0) return PDG_OK;
    const int64_t words = nh + (nh + 1) + 3 * np;
    if (words > ctx->hub_cap) {
        if (ctx->d_hub) PDG_HIP(ctx, hipFree(ctx->d_hub));
        ctx->d_hub = nullptr;
        ctx->hub_cap = 0;
        PDG_TRY(dalloc(ctx, (void **)&ctx->d_hub, words * 4));
        ctx->hub_cap = words;
    }
    const int64_t pd = np * ctx->CB * (ctx->QM - 1) * 64;
    if (pd > ctx->part_cap) {
        if (ctx->d_part) PDG_HIP(ctx, hipFree(ctx->d_part));
        ctx->d_part = nullptr;
        ctx->part_cap = 0;
        PDG_TRY(dalloc(ctx, (void **)&ctx->d_part, pd * 8));
        ctx->part_cap = pd;
    }
    std::vector<uint32_t> all;
    all.reserve(words);
    all.insert(all.end(), hn.begin(), hn.end());
    all.insert(all.end(), hp.begin(), hp.end());
    all.insert(all.end(), pn_node.begin(), pn_node.end());
    all.insert(all.end(), pf.begin(), pf.end());
    all.insert(all.end(), pn.begin(), pn.end());
    PDG_HIP(ctx, hipMemcpyAsync(ctx->d_hub, all.data(), words * 4, hipMemcpyHostToDevice,
                                ctx->stream));
    PDG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->nh = nh;
    ctx->np = np;
    ctx->hub_thr = kHubThreshold;
    return PDG_OK;
}

static void free_all(pdg_ctx *ctx)
{
    void *ps[] = {ctx->d_q,     ctx->d_lam,   ctx->d_x,     ctx->d_counts, ctx->d_src,
                  ctx->d_dst,   ctx->d_uid,   ctx->d_sq,    ctx->d_params, ctx->d_ipos,
                  ctx->d_off,   ctx->d_cnt,   ctx->d_pool,  ctx->d_rec_p,  ctx->d_rec_z,
                  ctx->d_flag,  ctx->d_scratch, ctx->d_base, ctx->d_hub, ctx->d_part};
    for (void *p : ps)
        if (p) (void)hipFree(p);
}

}  // namespace pdg

using namespace pdg;

// ======================================================================= ABI
extern "C" {

const char *pdg_last_error(const pdg_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : g_global_err.c_str();
}

pdg_status pdg_create(const pdg_config *cfg, int32_t device, void *stream, pdg_ctx **out)
{
    if (!cfg || !out) return fail(nullptr, PDG_EINVAL, "null argument");
    *out = nullptr;
    if (cfg->n_chains < 1 || cfg->n_chains > (1 << 26))
        return fail(nullptr, PDG_EINVAL, "n_chains must be in [1, 2^26]");
    if (cfg->q_max < 2 || cfg->q_max > 8) return fail(nullptr, PDG_EINVAL, "q_max must be in [2, 8]");
    if (cfg->node_capacity < 1 || cfg->edge_capacity < 1 || cfg->edge_capacity >= (1ll << 31))
        return fail(nullptr, PDG_EINVAL, "capacities must be >= 1 (edges < 2^31)");
    if (cfg->precision != PDG_PRECISION_F32 && cfg->precision != PDG_PRECISION_F64)
        return fail(nullptr, PDG_EINVAL, "precision must be PDG_PRECISION_F32 or _F64");
    if (cfg->reserved != 0 || cfg->burn_in < 0) return fail(nullptr, PDG_EINVAL, "bad config");
    if ((int64_t)cfg->node_capacity * cfg->n_chains > (1ll << 40))
        return fail(nullptr, PDG_ECAPACITY, "node_capacity * n_chains too large");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(nullptr, PDG_EINVAL, "no such HIP device");
    pdg_ctx *ctx = new (std::nothrow) pdg_ctx();
    if (!ctx) return fail(nullptr, PDG_ENOMEM, "host allocation failed");
    ctx->cfg = *cfg;
    ctx->device = device;
    ctx->stream = (hipStream_t)stream;
    ctx->QM = cfg->q_max;
    ctx->D = dim_d(ctx->QM);
    ctx->C = cfg->n_chains;
    ctx->LPI = choose_lpi(ctx->C);
    ctx->CB = (int)cdiv(ctx->C, ctx->LPI);
    ctx->RP = rec_len(ctx->QM);
    ctx->ZW = rec_words(ctx->QM, ctx->C);
    ctx->bbytes = block_bytes(ctx->QM);
    pdg_status s = PDG_OK;
    auto bail = [&](pdg_status code) {
        std::string m = ctx->err;
        free_all(ctx);
        delete ctx;
        g_global_err = m;
        return code;
    };
    if (hipSetDevice(device) != hipSuccess) return bail(fail(ctx, PDG_EHIP, "hipSetDevice failed"));
    const int64_t N = cfg->node_capacity, S = cfg->edge_capacity;
    const int64_t N4 = (N + 3) / 4 * 4;  // segment tables are read per node quad
    // slot arrays are read in groups of kDualEdgesPerWave slots
    const int64_t SP = (S + kDualEdgesPerWave - 1) / kDualEdgesPerWave * kDualEdgesPerWave;
    if ((s = dalloc(ctx, (void **)&ctx->d_q, N)) ||
        (s = dalloc(ctx, (void **)&ctx->d_lam, N * ctx->QM * 8)) ||
        (s = dalloc(ctx, (void **)&ctx->d_x, N * ctx->C)) ||
        (s = dalloc(ctx, (void **)&ctx->d_counts, N4 * ctx->QM * 4)) ||
        (s = dalloc(ctx, (void **)&ctx->d_base, N4 * ctx->QM * 8)) ||
        (s = dalloc(ctx, (void **)&ctx->d_src, SP * 4)) ||
        (s = dalloc(ctx, (void **)&ctx->d_dst, SP * 4)) ||
        (s = dalloc(ctx, (void **)&ctx->d_uid, SP * 8)) ||
        (s = dalloc(ctx, (void **)&ctx->d_sq, SP)) ||
        (s = dalloc(ctx, (void **)&ctx->d_params, SP * ctx->bbytes)) ||
        (s = dalloc(ctx, (void **)&ctx->d_ipos, SP * 8)) ||
        (s = dalloc(ctx, (void **)&ctx->d_off, N4 * 4)) ||
        (s = dalloc(ctx, (void **)&ctx->d_cnt, N4 * 4)) ||
        (s = dalloc(ctx, (void **)&ctx->d_flag, 64)))
        return bail(s);
    if (hipMemsetAsync(ctx->d_uid, 0, SP * 8, ctx->stream) != hipSuccess ||
        hipMemsetAsync(ctx->d_src, 0, SP * 4, ctx->stream) != hipSuccess ||
        hipMemsetAsync(ctx->d_dst, 0, SP * 4, ctx->stream) != hipSuccess ||
        hipMemsetAsync(ctx->d_sq, 0, SP, ctx->stream) != hipSuccess ||
        hipMemsetAsync(ctx->d_ipos, 0, SP * 8, ctx->stream) != hipSuccess ||
        hipMemsetAsync(ctx->d_off, 0, N4 * 4, ctx->stream) != hipSuccess ||
        hipMemsetAsync(ctx->d_cnt, 0, N4 * 4, ctx->stream) != hipSuccess ||
        hipMemsetAsync(ctx->d_counts, 0, N4 * ctx->QM * 4, ctx->stream) != hipSuccess ||
        hipMemsetAsync(ctx->d_base, 0, N4 * ctx->QM * 8, ctx->stream) != hipSuccess ||
        hipMemsetAsync(ctx->d_x, 0, N * ctx->C, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
        return bail(fail(ctx, PDG_EHIP, "initial clear failed"));
    Store &st = ctx->st;
    try {
        st.S = S;
        st.slot.assign(S, SlotRec{0, 0, 0, 0, 0, 0, 0});
        st.free_stack.resize(S);
        for (int64_t j = 0; j < S; ++j) st.free_stack[j] = (int32_t)(S - 1 - j);
    } catch (...) {
        return bail(fail(ctx, PDG_ENOMEM, "host allocation failed"));
    }
    *out = ctx;
    return PDG_OK;
}

pdg_status pdg_destroy(pdg_ctx *ctx)
{
    if (!ctx) return PDG_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    free_all(ctx);
    delete ctx;
    return PDG_OK;
}

pdg_status pdg_set_nodes(pdg_ctx *ctx, int64_t n, const int32_t *d_q, const void *d_log_unary)
{
    if (!ctx) return fail(nullptr, PDG_EINVAL, "null context");
    if (ctx->nodes_set) return fail(ctx, PDG_ESTATE, "nodes already set");
    if (n < 1 || n > ctx->cfg.node_capacity) return fail(ctx, PDG_EINVAL, "n out of range");
    if (!d_q || !d_log_unary) return fail(ctx, PDG_EINVAL, "null pointer");
    PDG_TRY(set_dev(ctx));
    PDG_TRY(clear_flag(ctx));
    if (ctx->cfg.precision == PDG_PRECISION_F64)
        k_set_nodes<double><<<grid_for(n), 256, 0, ctx->stream>>>(
            n, ctx->QM, d_q, static_cast<const double *>(d_log_unary), ctx->d_q, ctx->d_lam,
            ctx->d_flag);
    else
        k_set_nodes<float><<<grid_for(n), 256, 0, ctx->stream>>>(
            n, ctx->QM, d_q, static_cast<const float *>(d_log_unary), ctx->d_q, ctx->d_lam,
            ctx->d_flag);
    PDG_HIP(ctx, hipGetLastError());
    uint32_t bad = 0;
    PDG_TRY(read_flag(ctx, &bad));
    if (bad & 2u) return fail(ctx, PDG_EINVAL, "q_i outside [2, q_max]");
    if (bad & 1u) return fail(ctx, PDG_ENONPOS, "non-finite log unary");
    {
        std::vector<int32_t> hq(n);
        PDG_HIP(ctx, hipMemcpyAsync(hq.data(), d_q, n * 4, hipMemcpyDeviceToHost, ctx->stream));
        PDG_HIP(ctx, hipStreamSynchronize(ctx->stream));
        ctx->uq = std::all_of(hq.begin(), hq.end(), [&](int32_t v) { return v == ctx->QM; });
    }
    Store &st = ctx->st;
    st.node.assign(n, NodeRec{0, 0, 0, 0});
    st.mark.assign(n, 0);
    ctx->n = n;
    PDG_HIP(ctx, hipMemsetAsync(ctx->d_off, 0, n * 4, ctx->stream));
    PDG_HIP(ctx, hipMemsetAsync(ctx->d_cnt, 0, n * 4, ctx->stream));
    // no incidences yet: base = lam
    PDG_HIP(ctx, hipMemcpyAsync(ctx->d_base, ctx->d_lam, n * ctx->QM * 8, hipMemcpyDeviceToDevice,
                                ctx->stream));
    PDG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->nodes_set = true;
    return PDG_OK;
}

pdg_status pdg_insert_edges(pdg_ctx *ctx, int64_t m, const int32_t *d_src, const int32_t *d_dst,
                            const void *d_log_phi, uint64_t *d_uid_out)
{
    if (!ctx) return fail(nullptr, PDG_EINVAL, "null context");
    if (!ctx->nodes_set) return fail(ctx, PDG_ESTATE, "pdg_set_nodes first");
    if (ctx->phase != 0) return fail(ctx, PDG_ESTATE, "edits only between sweeps");
    if (m < 0) return fail(ctx, PDG_EINVAL, "m < 0");
    if (m == 0) return PDG_OK;
    if (!d_src || !d_dst || !d_log_phi) return fail(ctx, PDG_EINVAL, "null pointer");
    PDG_TRY(set_dev(ctx));
    Store &st = ctx->st;
    if ((int64_t)st.free_stack.size() < m) return fail(ctx, PDG_ECAPACITY, "edge capacity exhausted");
    std::vector<int32_t> hs(m), hd(m);
    PDG_HIP(ctx, hipMemcpyAsync(hs.data(), d_src, m * 4, hipMemcpyDeviceToHost, ctx->stream));
    PDG_HIP(ctx, hipMemcpyAsync(hd.data(), d_dst, m * 4, hipMemcpyDeviceToHost, ctx->stream));
    PDG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int64_t k = 0; k < m; ++k) {
        if (hs[k] < 0 || hs[k] >= ctx->n || hd[k] < 0 || hd[k] >= ctx->n)
            return fail(ctx, PDG_EINVAL, "edge endpoint out of range");
        if (hs[k] == hd[k]) return fail(ctx, PDG_EINVAL, "self-loop is not a pairwise factor");
    }
    for (int64_t k = 0; k < m; ++k)
        if (st.slot[st.free_stack[st.free_stack.size() - 1 - k]].gen == 0xFFFFFFFFu)
            return fail(ctx, PDG_ECAPACITY, "uid space of a slot exhausted");
    // tables must be finite before anything changes
    PDG_TRY(clear_flag(ctx));
    launch_check(ctx->QM, ctx->cfg.precision == PDG_PRECISION_F64, m, d_src, d_dst, ctx->d_q,
                 d_log_phi, ctx->d_flag, ctx->stream);
    PDG_HIP(ctx, hipGetLastError());
    uint32_t bad = 0;
    PDG_TRY(read_flag(ctx, &bad));
    if (bad) return fail(ctx, PDG_ENONPOS, "non-finite log factor entry");

    // slots and uids
    std::vector<int32_t> slots(m);
    std::vector<uint64_t> uids(m);
    const int64_t fs0 = (int64_t)st.free_stack.size();
    for (int64_t k = 0; k < m; ++k) {
        if (k + kAhead < m) prefetch_w(&st.slot[st.free_stack[fs0 - 1 - (k + kAhead)]]);
        const int32_t s = st.free_stack.back();
        st.free_stack.pop_back();
        st.slot[s].gen += 1;
        const uint64_t u = ((uint64_t)st.slot[s].gen << 32) | (uint32_t)s;
        slots[k] = s;
        uids[k] = u;
        st.slot[s].uid = u;
        st.slot[s].src = hs[k];
        st.slot[s].dst = hd[k];
        st.hwm = std::max<int64_t>(st.hwm, (int64_t)s + 1);
    }
    st.live += m;
    // incidence: room first (relocation or full compaction), then appends in batch order
    Patches P;
    std::vector<uint32_t> &need = st.mark;  // reset for the touched nodes before returning
    std::vector<int64_t> touched;
    try {
        touched.reserve(2 * m);
        for (int64_t k = 0; k < m; ++k) {
            if (k + kAhead < m) {
                prefetch_w(&need[hs[k + kAhead]]);
                prefetch_w(&need[hd[k + kAhead]]);
            }
            if (need[hs[k]]++ == 0) touched.push_back(hs[k]);
            if (need[hd[k]]++ == 0) touched.push_back(hd[k]);
        }
    } catch (...) {
        for (int64_t k = 0; k < m; ++k) need[hs[k]] = need[hd[k]] = 0;
        return fail(ctx, PDG_ENOMEM, "host allocation failed");
    }
    struct Reset {
        std::vector<uint32_t> &v;
        const std::vector<int64_t> &idx;
        ~Reset() { for (int64_t i : idx) v[i] = 0; }
    } reset_need{need, touched};
    uint64_t room = 0;
    for (size_t k = 0; k < touched.size(); ++k) {
        if (k + kAhead < touched.size()) prefetch_w(&st.node[touched[k + kAhead]]);
        const int64_t i = touched[k];
        if (st.node[i].cnt + need[i] > st.node[i].cap) {
            const uint32_t want = st.node[i].nlive + need[i];
            room += want + slack_for(want);
        }
    }
    if ((uint64_t)st.pool_top + room > (uint64_t)st.pool.size()) {
        PDG_TRY(full_compact(ctx, need, P));
    } else {
        for (int64_t i : touched)
            if (st.node[i].cnt + need[i] > st.node[i].cap) relocate(ctx, i, need[i], P);
    }
    P.idx.reserve(P.idx.size() + 2 * m);
    P.val.reserve(P.val.size() + 2 * m);
    P.ip_key.reserve(P.ip_key.size() + 2 * m);
    P.ip_val.reserve(P.ip_val.size() + 2 * m);
    for (int64_t k = 0; k < m; ++k) {
        if (k + kAhead < m) {  // node headers ahead, then the pool lines they point at
            prefetch_w(&st.node[hs[k + kAhead]]);
            prefetch_w(&st.node[hd[k + kAhead]]);
        }
        if (k + kAhead / 2 < m) {
            const NodeRec &a = st.node[hs[k + kAhead / 2]], &b = st.node[hd[k + kAhead / 2]];
            prefetch_w(st.pool.data() + a.off + a.cnt);
            prefetch_w(st.pool.data() + b.off + b.cnt);
        }
        append(ctx, hs[k], ((uint32_t)slots[k] << 1) | 0u, P);
        append(ctx, hd[k], ((uint32_t)slots[k] << 1) | 1u, P);
    }
    // device: incidence structure and records (moves, ipos), then slot
    // arrays, decomposition of the new tables, and their records
    PDG_TRY(upload(ctx, P, touched));
    PDG_TRY(rebuild_hubs(ctx));
    const int64_t nn = (int64_t)touched.size();
    std::vector<uint32_t> hnodes(touched.begin(), touched.end());
    void *s;
    PDG_TRY(scratch(ctx, 8 * m + 4 * m * 3 + 4 * nn + 64, &s));
    uint64_t *du = (uint64_t *)s;
    int32_t *dslot = (int32_t *)(du + m), *dqs = dslot + m, *dqd = dqs + m;
    uint32_t *dnodes = (uint32_t *)(dqd + m);
    PDG_HIP(ctx, hipMemcpyAsync(dnodes, hnodes.data(), nn * 4, hipMemcpyHostToDevice, ctx->stream));
    PDG_HIP(ctx, hipMemcpyAsync(du, uids.data(), m * 8, hipMemcpyHostToDevice, ctx->stream));
    PDG_HIP(ctx, hipMemcpyAsync(dslot, slots.data(), m * 4, hipMemcpyHostToDevice, ctx->stream));
    k_slot_write<<<grid_for(m), 256, 0, ctx->stream>>>(m, dslot, d_src, d_dst, du, ctx->d_q,
                                                       ctx->d_src, ctx->d_dst, ctx->d_uid,
                                                       ctx->d_sq, dqs, dqd, d_uid_out);
    PDG_HIP(ctx, hipGetLastError());
    PDG_TRY(clear_flag(ctx));
    launch_decompose(ctx->QM, ctx->cfg.precision == PDG_PRECISION_F64, m, dqs, dqd, d_log_phi,
                     dslot, ctx->d_params, ctx->d_flag, ctx->stream);
    PDG_HIP(ctx, hipGetLastError());
    k_write_records<<<grid_for(m * ctx->RP), 256, 0, ctx->stream>>>(
        m, ctx->QM, dslot, ctx->d_sq, ctx->d_params, ctx->d_ipos, ctx->d_rec_p);
    launch_node_base(ctx, nn, dnodes);
    PDG_HIP(ctx, hipGetLastError());
    PDG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return PDG_OK;
}

pdg_status pdg_remove_edges(pdg_ctx *ctx, int64_t m, const uint64_t *d_uid)
{
    if (!ctx) return fail(nullptr, PDG_EINVAL, "null context");
    if (ctx->phase != 0) return fail(ctx, PDG_ESTATE, "edits only between sweeps");
    if (m < 0) return fail(ctx, PDG_EINVAL, "m < 0");
    if (m == 0) return PDG_OK;
    if (!d_uid) return fail(ctx, PDG_EINVAL, "null pointer");
    PDG_TRY(set_dev(ctx));
    Store &st = ctx->st;
    std::vector<uint64_t> hu(m);
    PDG_HIP(ctx, hipMemcpyAsync(hu.data(), d_uid, m * 8, hipMemcpyDeviceToHost, ctx->stream));
    PDG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    std::vector<int32_t> slots(m);
    for (int64_t k = 0; k < m; ++k) {
        if (k + kAhead < m) {
            const int64_t sa = (int64_t)(hu[k + kAhead] & 0xFFFFFFFFull);
            if (sa < st.S) prefetch_w(&st.slot[sa]);
        }
        const uint64_t u = hu[k];
        const int64_t s = (int64_t)(u & 0xFFFFFFFFull);
        if (u == 0 || s >= st.S || st.slot[s].uid != u) {
            for (int64_t j = 0; j < k; ++j) st.slot[slots[j]].uid = hu[j];
            return fail(ctx, PDG_ENOTFOUND, "uid " + std::to_string(u) + " is not a live edge");
        }
        slots[k] = (int32_t)s;
        st.slot[s].uid = 0;  // also catches a uid repeated within the batch
    }
    Patches P;
    std::vector<int64_t> touched;
    std::vector<uint32_t> recs, hnodes;
    recs.reserve(2 * m);
    hnodes.reserve(2 * m);
    P.idx.reserve(2 * m);
    P.val.reserve(2 * m);
    st.free_stack.reserve(st.free_stack.size() + m);
    for (int64_t k = 0; k < m; ++k) {
        if (k + kAhead < m) {  // the slot lines were fetched by the validation loop
            const SlotRec &r = st.slot[slots[k + kAhead]];
            prefetch_w(&st.node[r.src]);
            prefetch_w(&st.node[r.dst]);
        }
        if (k + kAhead / 2 < m) {
            const SlotRec &r = st.slot[slots[k + kAhead / 2]];
            prefetch_w(st.pool.data() + st.node[r.src].off + r.pos0);
            prefetch_w(st.pool.data() + st.node[r.dst].off + r.pos1);
        }
        const int32_t s = slots[k];
        const int32_t a = st.slot[s].src, b = st.slot[s].dst;
        const uint32_t ia = st.node[a].off + st.slot[s].pos0, ib = st.node[b].off + st.slot[s].pos1;
        st.pool[ia] = kTomb;
        st.pool[ib] = kTomb;
        P.idx.push_back(ia);
        P.val.push_back(kTomb);
        P.idx.push_back(ib);
        P.val.push_back(kTomb);
        recs.push_back(ia);
        recs.push_back(ib);
        hnodes.push_back((uint32_t)a);
        hnodes.push_back((uint32_t)b);
        st.node[a].nlive--;
        st.node[b].nlive--;
        st.free_stack.push_back(s);
    }
    st.live -= m;
    PDG_TRY(upload(ctx, P, touched));
    {  // distinct endpoints, first-seen order
        size_t w = 0;
        for (size_t k = 0; k < hnodes.size(); ++k)
            if (st.mark[hnodes[k]]++ == 0) hnodes[w++] = hnodes[k];
        hnodes.resize(w);
        for (uint32_t i : hnodes) st.mark[i] = 0;
    }
    const int64_t nn = (int64_t)hnodes.size();
    void *sp;
    PDG_TRY(scratch(ctx, 4 * m + 8 * m + 4 * nn + 768, &sp));
    int32_t *dsl = (int32_t *)sp;
    uint32_t *drec = (uint32_t *)((char *)sp + ((4 * m + 255) / 256) * 256);
    uint32_t *dnodes = (uint32_t *)((char *)drec + ((8 * m + 255) / 256) * 256);
    PDG_HIP(ctx, hipMemcpyAsync(dsl, slots.data(), m * 4, hipMemcpyHostToDevice, ctx->stream));
    PDG_HIP(ctx, hipMemcpyAsync(drec, recs.data(), 2 * m * 4, hipMemcpyHostToDevice, ctx->stream));
    PDG_HIP(ctx, hipMemcpyAsync(dnodes, hnodes.data(), nn * 4, hipMemcpyHostToDevice, ctx->stream));
    k_slot_clear<<<grid_for(m), 256, 0, ctx->stream>>>(m, dsl, ctx->d_uid);
    k_clear_records<<<grid_for(2 * m * ctx->RP), 256, 0, ctx->stream>>>(2 * m, ctx->RP, drec,
                                                                       ctx->d_rec_p);
    launch_node_base(ctx, nn, dnodes);
    PDG_HIP(ctx, hipGetLastError());
    PDG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return PDG_OK;
}

pdg_status pdg_num_edges(pdg_ctx *ctx, int64_t *h_live)
{
    if (!ctx || !h_live) return fail(ctx, PDG_EINVAL, "null argument");
    *h_live = ctx->st.live;
    return PDG_OK;
}

pdg_status pdg_live_uids(pdg_ctx *ctx, uint64_t *d_uid_out)
{
    if (!ctx || !d_uid_out) return fail(ctx, PDG_EINVAL, "null argument");
    PDG_TRY(set_dev(ctx));
    std::vector<uint64_t> out;
    out.reserve(ctx->st.live);
    for (int64_t s = 0; s < ctx->st.hwm; ++s)
        if (ctx->st.slot[s].uid) out.push_back(ctx->st.slot[s].uid);
    if (!out.empty()) {
        PDG_HIP(ctx, hipMemcpyAsync(d_uid_out, out.data(), out.size() * 8, hipMemcpyHostToDevice,
                                    ctx->stream));
        PDG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }
    return PDG_OK;
}

pdg_status pdg_params_layout(int32_t q_max, int64_t *h_bytes, int64_t *h_off_sign,
                             int64_t *h_off_thr, int64_t *h_off_h, int64_t *h_off_c0)
{
    if (q_max < 2 || q_max > 8) return fail(nullptr, PDG_EINVAL, "q_max must be in [2, 8]");
    if (h_bytes) *h_bytes = block_bytes(q_max);
    if (h_off_sign) *h_off_sign = 0;
    if (h_off_thr) *h_off_thr = off_thr(q_max);
    if (h_off_h) *h_off_h = off_h(q_max);
    if (h_off_c0) *h_off_c0 = off_c0(q_max);
    return PDG_OK;
}

pdg_status pdg_decompose(int64_t m, int32_t q_max, const int32_t *d_qs, const int32_t *d_qd,
                         const void *d_log_phi, int32_t precision, void *d_params_out, void *stream)
{
    if (q_max < 2 || q_max > 8) return fail(nullptr, PDG_EINVAL, "q_max must be in [2, 8]");
    if (m < 0) return fail(nullptr, PDG_EINVAL, "m < 0");
    if (m == 0) return PDG_OK;
    if (!d_qs || !d_qd || !d_log_phi || !d_params_out) return fail(nullptr, PDG_EINVAL, "null pointer");
    if (precision != PDG_PRECISION_F32 && precision != PDG_PRECISION_F64)
        return fail(nullptr, PDG_EINVAL, "bad precision");
    hipStream_t s = (hipStream_t)stream;
    uint32_t *bad = nullptr;
    if (hipMalloc((void **)&bad, 4) != hipSuccess) return fail(nullptr, PDG_ENOMEM, "hipMalloc failed");
    k_fill_u32<<<1, 64, 0, s>>>(bad, 1, 0u);
    launch_decompose(q_max, precision == PDG_PRECISION_F64, m, d_qs, d_qd, d_log_phi, nullptr,
                     (uint8_t *)d_params_out, bad, s);
    uint32_t hb = 0;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&hb, bad, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(bad);
    if (e != hipSuccess) return fail(nullptr, PDG_EHIP, std::string("decompose: ") + hipGetErrorString(e));
    if (hb & 2u) return fail(nullptr, PDG_EINVAL, "a state count is outside [2, q_max]");
    if (hb) return fail(nullptr, PDG_ENONPOS, "non-finite log factor entry");
    return PDG_OK;
}

pdg_status pdg_init_chains(pdg_ctx *ctx)
{
    if (!ctx) return fail(nullptr, PDG_EINVAL, "null context");
    if (!ctx->nodes_set) return fail(ctx, PDG_ESTATE, "pdg_set_nodes first");
    PDG_TRY(set_dev(ctx));
    const int64_t nc = ctx->n * ctx->C;
    k_init<<<grid_for(nc), 256, 0, ctx->stream>>>(ctx->n, ctx->C, ctx->d_q, ctx->d_x,
                                                  (uint32_t)ctx->cfg.seed,
                                                  (uint32_t)(ctx->cfg.seed >> 32));
    PDG_HIP(ctx, hipGetLastError());
    ctx->t = 0;
    ctx->phase = 0;
    return PDG_OK;
}

pdg_status pdg_set_state(pdg_ctx *ctx, const uint8_t *d_x)
{
    if (!ctx || !d_x) return fail(ctx, PDG_EINVAL, "null argument");
    if (!ctx->nodes_set) return fail(ctx, PDG_ESTATE, "pdg_set_nodes first");
    PDG_TRY(set_dev(ctx));
    PDG_HIP(ctx, hipMemcpyAsync(ctx->d_x, d_x, ctx->n * ctx->C, hipMemcpyDeviceToDevice, ctx->stream));
    return PDG_OK;
}

pdg_status pdg_get_state(pdg_ctx *ctx, uint8_t *d_x_out)
{
    if (!ctx || !d_x_out) return fail(ctx, PDG_EINVAL, "null argument");
    PDG_TRY(set_dev(ctx));
    PDG_HIP(ctx, hipMemcpyAsync(d_x_out, ctx->d_x, ctx->n * ctx->C, hipMemcpyDeviceToDevice, ctx->stream));
    return PDG_OK;
}

pdg_status pdg_get_sweep(pdg_ctx *ctx, int64_t *h_t)
{
    if (!ctx || !h_t) return fail(ctx, PDG_EINVAL, "null argument");
    *h_t = ctx->t;
    return PDG_OK;
}

pdg_status pdg_set_sweep(pdg_ctx *ctx, int64_t t)
{
    if (!ctx) return fail(nullptr, PDG_EINVAL, "null context");
    if (t < 0 || t >= 0xFFFFFFFFll) return fail(ctx, PDG_EINVAL, "sweep counter out of range");
    if (ctx->phase != 0) return fail(ctx, PDG_ESTATE, "between sweeps only");
    ctx->t = t;
    return PDG_OK;
}

pdg_status pdg_dual_phase(pdg_ctx *ctx)
{
    if (!ctx) return fail(nullptr, PDG_EINVAL, "null context");
    if (!ctx->nodes_set) return fail(ctx, PDG_ESTATE, "pdg_set_nodes first");
    if (ctx->phase != 0) return fail(ctx, PDG_ESTATE, "primal phase pending");
    if (ctx->t + 1 >= 0xFFFFFFFFll) return fail(ctx, PDG_ECAPACITY, "sweep counter exhausted");
    PDG_TRY(set_dev(ctx));
    ctx->t += 1;
    if (ctx->st.hwm > 0) {
        launch_dual(ctx, (uint32_t)ctx->t);
        PDG_HIP(ctx, hipGetLastError());
    }
    ctx->phase = 1;
    return PDG_OK;
}

pdg_status pdg_primal_phase(pdg_ctx *ctx)
{
    if (!ctx) return fail(nullptr, PDG_EINVAL, "null context");
    if (ctx->phase != 1) return fail(ctx, PDG_ESTATE, "dual phase first");
    const int count = ctx->t > ctx->cfg.burn_in ? 1 : 0;
    if (count && (uint64_t)(ctx->counted + 1) * (uint64_t)ctx->C > 0xFFFFFFFFull)
        return fail(ctx, PDG_ECAPACITY, "marginal counters would overflow; read and reset them");
    PDG_TRY(set_dev(ctx));
    launch_primal(ctx, (uint32_t)ctx->t, count);
    PDG_HIP(ctx, hipGetLastError());
    ctx->counted += count;
    ctx->phase = 0;
    return PDG_OK;
}

pdg_status pdg_sweep(pdg_ctx *ctx, int64_t n_sweeps)
{
    if (!ctx) return fail(nullptr, PDG_EINVAL, "null context");
    if (n_sweeps < 0) return fail(ctx, PDG_EINVAL, "n_sweeps < 0");
    for (int64_t k = 0; k < n_sweeps; ++k) {
        PDG_TRY(pdg_dual_phase(ctx));
        PDG_TRY(pdg_primal_phase(ctx));
    }
    return PDG_OK;
}

pdg_status pdg_get_duals(pdg_ctx *ctx, int64_t m, const uint64_t *d_uid, uint64_t *d_theta_out)
{
    if (!ctx) return fail(nullptr, PDG_EINVAL, "null context");
    if (m < 0) return fail(ctx, PDG_EINVAL, "m < 0");
    if (m == 0) return PDG_OK;
    if (!d_uid || !d_theta_out) return fail(ctx, PDG_EINVAL, "null pointer");
    PDG_TRY(set_dev(ctx));
    std::vector<uint64_t> hu(m);
    PDG_HIP(ctx, hipMemcpyAsync(hu.data(), d_uid, m * 8, hipMemcpyDeviceToHost, ctx->stream));
    PDG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    std::vector<int32_t> slots(m);
    for (int64_t k = 0; k < m; ++k) {
        const int64_t s = (int64_t)(hu[k] & 0xFFFFFFFFull);
        if (hu[k] == 0 || s >= ctx->st.S || ctx->st.slot[s].uid != hu[k])
            return fail(ctx, PDG_ENOTFOUND, "uid is not a live edge");
        slots[k] = (int32_t)s;
    }
    void *sp;
    PDG_TRY(scratch(ctx, 4 * m + 64, &sp));
    PDG_HIP(ctx, hipMemcpyAsync(sp, slots.data(), m * 4, hipMemcpyHostToDevice, ctx->stream));
    k_get_duals<<<grid_for(m * ctx->C), 256, 0, ctx->stream>>>(m, ctx->QM, make_graph(ctx),
                                                               (const int32_t *)sp, d_theta_out);
    PDG_HIP(ctx, hipGetLastError());
    PDG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return PDG_OK;
}

pdg_status pdg_get_marginals(pdg_ctx *ctx, double *d_out, int64_t *h_samples)
{
    if (!ctx || !d_out) return fail(ctx, PDG_EINVAL, "null argument");
    PDG_TRY(set_dev(ctx));
    const int64_t samples = ctx->counted * ctx->C;
    const double inv = samples ? 1.0 / (double)samples : 0.0;
    const int64_t nq = ctx->n * ctx->QM;
    k_marginals<<<grid_for(nq), 256, 0, ctx->stream>>>(nq, ctx->d_counts, inv, d_out);
    PDG_HIP(ctx, hipGetLastError());
    PDG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (h_samples) *h_samples = samples;
    return PDG_OK;
}

pdg_status pdg_get_counts(pdg_ctx *ctx, uint32_t *d_out, int64_t *h_samples)
{
    if (!ctx || !d_out) return fail(ctx, PDG_EINVAL, "null argument");
    PDG_TRY(set_dev(ctx));
    PDG_HIP(ctx, hipMemcpyAsync(d_out, ctx->d_counts, ctx->n * ctx->QM * 4, hipMemcpyDeviceToDevice,
                                ctx->stream));
    PDG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (h_samples) *h_samples = ctx->counted * ctx->C;
    return PDG_OK;
}

pdg_status pdg_reset_marginals(pdg_ctx *ctx)
{
    if (!ctx) return fail(nullptr, PDG_EINVAL, "null context");
    PDG_TRY(set_dev(ctx));
    const int64_t nq = ctx->n * ctx->QM;
    k_fill_u32<<<grid_for(nq), 256, 0, ctx->stream>>>(ctx->d_counts, nq, 0u);
    PDG_HIP(ctx, hipGetLastError());
    ctx->counted = 0;
    return PDG_OK;
}

pdg_status pdg_sync(pdg_ctx *ctx)
{
    if (!ctx) return fail(nullptr, PDG_EINVAL, "null context");
    PDG_TRY(set_dev(ctx));
    PDG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    PDG_HIP(ctx, hipGetLastError());
    return PDG_OK;
}

}  // extern "C"

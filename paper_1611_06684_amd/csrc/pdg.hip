// libpdg: host runtime and C ABI of the primal-dual Gibbs sweep (include/pdg.h).
//
// The context owns every device buffer.  Sweeps are two kernels per sweep on
// the caller's stream.  Edge edits run as kernels too (pdg_store.hpp): a
// device free-slot stack with generation-tagged uids and per-node incidence
// segments with slack, so an edit batch costs O(batch) plus an occasional
// segment relocation; no colouring and no rebuild of the incidence lists is
// ever needed (the abstract, Sec. 1 and Sec. 6 of the paper motivate the
// method by exactly this setting).  The host only reads back a few counters
// (EditSummary) to size launches and report errors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>
#include <mutex>
#include <string>
#include <vector>

#include <hipcub/hipcub.hpp>

#include "pdg.h"
#include "pdg_view.hpp"
#include "pdg_kernels.hpp"
#include "pdg_store.hpp"

namespace pdg {

static thread_local std::string g_global_err;

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
    uint8_t *d_dparams = nullptr;  // [slot] sign word and thresholds of the block (thr_bytes)
    void *d_lphi = nullptr;  // [slot][QM][QM] log tables as given (float or double)
    uint32_t *d_ipos = nullptr;
    uint32_t *d_off = nullptr, *d_cnt = nullptr;
    uint32_t *d_pool = nullptr;
    double *d_rec_p = nullptr;
    uint32_t *d_rec_z = nullptr;
    int64_t dev_pool_cap = 0;
    // edge store (device side in pdg_store.hpp; the host keeps these scalars)
    int64_t S = 0;         // edge slots
    int64_t ftop = 0;      // height of the free-slot stack
    int64_t live = 0;      // live edges
    int64_t hwm = 0;       // slots [0, hwm) may be live
    int64_t pool_top = 0;  // first pool entry no segment uses
    int32_t *d_free = nullptr;
    uint32_t *d_gen = nullptr, *d_claim = nullptr;
    uint32_t *d_cap = nullptr, *d_nlive = nullptr, *d_mark = nullptr;
    pdg::EditSummary *d_sum = nullptr;
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
    // node order of the chain-major primal (nodes by record count, largest
    // first; rebuilt with the hub table)
    uint32_t *d_order = nullptr;
    bool order_set = false;
    int64_t part_cap = 0;        // doubles
    bool broken = false;         // an edit failed after it began to change the store
    void *d_static = nullptr;    // this device's copy of the static workspace (pdg_log_v_noalloc)
    uint64_t gen = 0;            // edge-store generation: advanced by every edit
    // launch parameters (pdg_tune / pdg_set_tuning): edges per wave of the
    // 33+-chain dual, item groups per wave of the binary dual, hub threshold
    // (0: hubs not split) and records per hub piece
    int32_t tune_e64 = 4, tune_ebin = 4;
    uint32_t tune_hub_thr = 256, tune_piece = 128;
    bool replay = false;         // launches are being captured for replay (device counter)
    std::string err;
};

// Static workspace of pdg_log_v_noalloc (callers that cannot allocate): every
// device the library runs on holds its own copy until the process ends.  Host
// code never uses the name itself; each context keeps this device's address of
// it, taken once per device when the first context is created there.
constexpr int64_t kStaticScratchBytes = 64ll << 20;
static __device__ __align__(256) double scratch[kStaticScratchBytes / 8];
static std::mutex g_static_mu;
static void *g_static_addr[256];

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

static pdg_status ctx_scratch(pdg_ctx *ctx, int64_t bytes, void **out)
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
    if (ctx->broken)
        return fail(ctx, PDG_ESTATE,
                    "an earlier edit failed while it was changing the edge store; destroy the context");
    PDG_HIP(ctx, hipSetDevice(ctx->device));
    return PDG_OK;
}

pdg_status report(pdg_ctx *ctx, pdg_status code, const std::string &msg)
{
    return fail(ctx, code, msg);
}

pdg_status ctx_view(pdg_ctx *ctx, CtxView *v)
{
    if (!ctx) return fail(nullptr, PDG_EINVAL, "null context");
    if (!ctx->nodes_set) return fail(ctx, PDG_ESTATE, "pdg_set_nodes first");
    PDG_TRY(set_dev(ctx));
    *v = CtxView{ctx->device, ctx->stream, ctx->d_x,          ctx->d_q,
                 ctx->n,      ctx->C,      ctx->QM,           ctx->cfg.precision,
                 ctx->cfg.seed, ctx->phase, ctx->d_rec_p,      ctx->d_rec_z,
                 ctx->d_off,  ctx->d_cnt,  ctx->d_base,       ctx->RP,
                 ctx->ZW};
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
    g.dparams = ctx->d_dparams;
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
    g.hwm = ctx->hwm;
    g.C = ctx->C;
    g.CB = (int32_t)cdiv(ctx->C, 64);
    g.heavy = ctx->hub_thr;
    g.order = ctx->order_set ? ctx->d_order : nullptr;
    g.k0 = (uint32_t)ctx->cfg.seed;
    g.k1 = (uint32_t)(ctx->cfg.seed >> 32);
    g.rk = make_round_keys(ctx->cfg.seed);
    // while sweeps are captured for replay the kernels read the sweep counter
    // from word 8 of the flag block, which the captured tick kernel advances
    g.tsrc = ctx->replay ? ctx->d_flag + 8 : nullptr;
    g.burn = ctx->cfg.burn_in;
    return g;
}

// ------------------------------------------------------------- kernel dispatch
template <int QM, bool UQ, int E>
static void dual64_e(const Graph &g, uint32_t t, int CB, hipStream_t s)
{
    const int64_t waves = cdiv(g.hwm, E) * CB;
    k_dual64<QM, UQ, E><<<grid_for(waves * 64), 256, 0, s>>>(g, t);
}

template <int LPI, bool UQ, int E>
static void dual_bin_e(const Graph &g, uint32_t t, hipStream_t s)
{
    constexpr int P = 64 / LPI;
    const int64_t waves = cdiv(cdiv(g.hwm, P), E);
    k_dual_bin<LPI, UQ, E><<<grid_for(waves * 64), 256, 0, s>>>(g, t);
}

template <int QM, int LPI, bool UQ>
static void launch_dual_t(const Graph &g, uint32_t t, int CB, hipStream_t s, int e64, int ebin)
{
    if constexpr (LPI == 64) {
        switch (e64) {
        case 2: dual64_e<QM, UQ, 2>(g, t, CB, s); break;
        case 8: dual64_e<QM, UQ, 8>(g, t, CB, s); break;
        default: dual64_e<QM, UQ, 4>(g, t, CB, s); break;
        }
    } else if constexpr (QM == 2 && (LPI == 8 || LPI == 16)) {
        switch (ebin) {
        case 2: dual_bin_e<LPI, UQ, 2>(g, t, s); break;
        case 8: dual_bin_e<LPI, UQ, 8>(g, t, s); break;
        default: dual_bin_e<LPI, UQ, 4>(g, t, s); break;
        }
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
        const int64_t waves = cdiv(g.n, 4);  // one quad per wave, record groups split the records
        if constexpr (QM >= 6)  // chain-major dual words (zc_layout)
            k_primal32z<QM, UQ, E64><<<grid_for(waves * 64), 256, 0, s>>>(g, t, count);
        else
            k_primal32<QM, UQ, E64><<<grid_for(waves * 64), 256, 0, s>>>(g, t, count);
    } else if constexpr ((LPI == 8 || LPI == 16) && QM >= 3) {
        // records of 4 or more entries: staged once per wave (binary records
        // are one word and one double; there the plain form is as fast)
        const int64_t waves = cdiv(cdiv(g.n, 4), P) * CB;
        k_primal_st<QM, LPI, UQ, E64><<<grid_for(waves * 64), 256, 0, s>>>(g, t, count);
    } else {
        const int64_t waves = cdiv(cdiv(g.n, 4), P) * CB;
        k_primal<QM, LPI, UQ, E64><<<grid_for(waves * 64), 256, 0, s>>>(g, t, count);
    }
}

template <int QM, bool UQ>
static void dual_q(int lpi, const Graph &g, uint32_t t, int CB, hipStream_t s, int e64, int ebin)
{
    switch (lpi) {
    case 1: launch_dual_t<QM, 1, UQ>(g, t, CB, s, e64, ebin); break;
    case 8: launch_dual_t<QM, 8, UQ>(g, t, CB, s, e64, ebin); break;
    case 16: launch_dual_t<QM, 16, UQ>(g, t, CB, s, e64, ebin); break;
    case 32: launch_dual_t<QM, 32, UQ>(g, t, CB, s, e64, ebin); break;
    default: launch_dual_t<QM, 64, UQ>(g, t, CB, s, e64, ebin); break;
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
    case 2: dual_q<2, UQ>(ctx->LPI, g, t, ctx->CB, ctx->stream, ctx->tune_e64, ctx->tune_ebin); break;
    case 3: dual_q<3, UQ>(ctx->LPI, g, t, ctx->CB, ctx->stream, ctx->tune_e64, ctx->tune_ebin); break;
    case 4: dual_q<4, UQ>(ctx->LPI, g, t, ctx->CB, ctx->stream, ctx->tune_e64, ctx->tune_ebin); break;
    case 5: dual_q<5, UQ>(ctx->LPI, g, t, ctx->CB, ctx->stream, ctx->tune_e64, ctx->tune_ebin); break;
    case 6: dual_q<6, UQ>(ctx->LPI, g, t, ctx->CB, ctx->stream, ctx->tune_e64, ctx->tune_ebin); break;
    case 7: dual_q<7, UQ>(ctx->LPI, g, t, ctx->CB, ctx->stream, ctx->tune_e64, ctx->tune_ebin); break;
    default: dual_q<8, UQ>(ctx->LPI, g, t, ctx->CB, ctx->stream, ctx->tune_e64, ctx->tune_ebin); break;
    }
}

static void launch_dual(pdg_ctx *ctx, uint32_t t)
{
    if (ctx->uq)
        launch_dual_u<true>(ctx, t);
    else
        launch_dual_u<false>(ctx, t);
}

template <int QM, int LPI, bool UQ, bool E64>
static void hubs_t(pdg_ctx *ctx, const Graph &g, uint32_t t, int count, int64_t wp, int64_t wf,
                   const uint32_t *hn, const uint32_t *hp, const uint32_t *pnode,
                   const uint32_t *pf, const uint32_t *pn)
{
    if constexpr (LPI == 32 && QM >= 6)
        k_hub_pieces_z<QM><<<grid_for(wp * 64), 256, 0, ctx->stream>>>(g, ctx->np, pnode, pf, pn,
                                                                        ctx->d_part);
    else
        k_hub_pieces<QM, LPI><<<grid_for(wp * 64), 256, 0, ctx->stream>>>(g, ctx->np, pnode, pf, pn,
                                                                          ctx->d_part);
    k_hub_finish<QM, UQ, E64, LPI><<<grid_for(wf * 64), 256, 0, ctx->stream>>>(
        g, ctx->nh, hn, hp, ctx->d_part, t, count);
}

template <int QM, bool UQ, bool E64>
static void launch_hubs_q(pdg_ctx *ctx, const Graph &g, uint32_t t, int count)
{
    const uint32_t *hn = ctx->d_hub, *hp = hn + ctx->nh, *pnode = hp + ctx->nh + 1;
    const uint32_t *pf = pnode + ctx->np, *pn = pf + ctx->np;
    const int64_t wp = ctx->np * ctx->CB, wf = ctx->nh * ctx->CB;
    switch (ctx->LPI) {
    case 1: hubs_t<QM, 1, UQ, E64>(ctx, g, t, count, wp, wf, hn, hp, pnode, pf, pn); break;
    case 8: hubs_t<QM, 8, UQ, E64>(ctx, g, t, count, wp, wf, hn, hp, pnode, pf, pn); break;
    case 16: hubs_t<QM, 16, UQ, E64>(ctx, g, t, count, wp, wf, hn, hp, pnode, pf, pn); break;
    case 32: hubs_t<QM, 32, UQ, E64>(ctx, g, t, count, wp, wf, hn, hp, pnode, pf, pn); break;
    default: hubs_t<QM, 64, UQ, E64>(ctx, g, t, count, wp, wf, hn, hp, pnode, pf, pn); break;
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

// Small graphs (up to 16 chains, at most kSmallWaves waves per phase): many
// sweeps in one launch of k_sweeps.
constexpr int64_t kSmallWaves = 32;
constexpr int32_t kSmallSweepsPerLaunch = 4096;

static bool small_waves(const pdg_ctx *ctx, int64_t *dw, int64_t *pw)
{
    // hubs are drawn by their own kernels, which the one-launch sweeps do not run
    if (ctx->LPI > 16 || ctx->nh > 0) return false;
    const int64_t P = 64 / ctx->LPI;
    *dw = cdiv(ctx->hwm, P) * ctx->CB;
    *pw = cdiv(cdiv(ctx->n, 4), P) * ctx->CB;
    return *dw <= kSmallWaves && *pw <= kSmallWaves;
}

template <int QM, int LPI, bool UQ, bool E64>
static void sweeps_t(pdg_ctx *ctx, uint32_t t0, int32_t n, int64_t dw, int64_t pw)
{
    const int64_t waves = std::max(dw, pw);
    const unsigned threads = (unsigned)std::min<int64_t>(1024, std::max<int64_t>(64, waves * 64));
    k_sweeps<QM, LPI, UQ, E64><<<1, threads, 0, ctx->stream>>>(
        make_graph(ctx), t0, n, ctx->cfg.burn_in, dw, pw);
}

template <int QM, bool UQ, bool E64>
static void sweeps_q(pdg_ctx *ctx, uint32_t t0, int32_t n, int64_t dw, int64_t pw)
{
    switch (ctx->LPI) {
    case 1: sweeps_t<QM, 1, UQ, E64>(ctx, t0, n, dw, pw); break;
    case 8: sweeps_t<QM, 8, UQ, E64>(ctx, t0, n, dw, pw); break;
    default: sweeps_t<QM, 16, UQ, E64>(ctx, t0, n, dw, pw); break;
    }
}

template <bool UQ, bool E64>
static void sweeps_u(pdg_ctx *ctx, uint32_t t0, int32_t n, int64_t dw, int64_t pw)
{
    switch (ctx->QM) {
    case 2: sweeps_q<2, UQ, E64>(ctx, t0, n, dw, pw); break;
    case 3: sweeps_q<3, UQ, E64>(ctx, t0, n, dw, pw); break;
    case 4: sweeps_q<4, UQ, E64>(ctx, t0, n, dw, pw); break;
    case 5: sweeps_q<5, UQ, E64>(ctx, t0, n, dw, pw); break;
    case 6: sweeps_q<6, UQ, E64>(ctx, t0, n, dw, pw); break;
    case 7: sweeps_q<7, UQ, E64>(ctx, t0, n, dw, pw); break;
    default: sweeps_q<8, UQ, E64>(ctx, t0, n, dw, pw); break;
    }
}

// Very small graphs (every edge-chain and node-chain pair one thread of one
// work-group, q_max <= 5, state within 64 KB of LDS): k_sweeps_lds.
static int64_t lds_bytes(const pdg_ctx *ctx)
{
    if (ctx->LPI > 16 || ctx->QM > 5) return -1;
    if (ctx->hwm * ctx->C > 1024 || ctx->n * ctx->C > 1024) return -1;
    const int64_t R = ctx->pool_top;  // bounds the entries in segments
    const int64_t b = R * ctx->D * (8 + ctx->C) + ctx->n * (4 * ctx->QM + 4 + ctx->C) + 64;
    return b <= 65536 ? b : -1;
}

template <int QM, bool UQ, bool E64>
static void sweeps_lds_q(pdg_ctx *ctx, uint32_t t0, int32_t n, int64_t bytes)
{
    if constexpr (QM <= 5) {
        const int64_t items = std::max(ctx->hwm, ctx->n) * ctx->C;
        const unsigned threads = (unsigned)std::min<int64_t>(1024, cdiv(items, 64) * 64);
        k_sweeps_lds<QM, UQ, E64><<<1, threads, (size_t)bytes, ctx->stream>>>(
            make_graph(ctx), t0, n, ctx->cfg.burn_in, (uint32_t)ctx->pool_top);
    }
}

template <bool UQ, bool E64>
static void sweeps_lds_u(pdg_ctx *ctx, uint32_t t0, int32_t n, int64_t bytes)
{
    switch (ctx->QM) {
    case 2: sweeps_lds_q<2, UQ, E64>(ctx, t0, n, bytes); break;
    case 3: sweeps_lds_q<3, UQ, E64>(ctx, t0, n, bytes); break;
    case 4: sweeps_lds_q<4, UQ, E64>(ctx, t0, n, bytes); break;
    default: sweeps_lds_q<5, UQ, E64>(ctx, t0, n, bytes); break;
    }
}

static void launch_sweeps(pdg_ctx *ctx, uint32_t t0, int32_t n, int64_t dw, int64_t pw)
{
    const int64_t bytes = lds_bytes(ctx);
    if (bytes > 0) {
        const bool e64 = ctx->cfg.precision == PDG_PRECISION_F64;
        if (ctx->uq) {
            if (e64) sweeps_lds_u<true, true>(ctx, t0, n, bytes);
            else sweeps_lds_u<true, false>(ctx, t0, n, bytes);
        } else {
            if (e64) sweeps_lds_u<false, true>(ctx, t0, n, bytes);
            else sweeps_lds_u<false, false>(ctx, t0, n, bytes);
        }
        return;
    }
    const bool e64 = ctx->cfg.precision == PDG_PRECISION_F64;
    if (ctx->uq) {
        if (e64) sweeps_u<true, true>(ctx, t0, n, dw, pw);
        else sweeps_u<true, false>(ctx, t0, n, dw, pw);
    } else {
        if (e64) sweeps_u<false, true>(ctx, t0, n, dw, pw);
        else sweeps_u<false, false>(ctx, t0, n, dw, pw);
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

// Check of an insert batch before anything changes (k_check_insert).
template <int QM>
static void check_insert_q(pdg_ctx *ctx, int64_t m, const int32_t *s, const int32_t *d,
                           const void *phi)
{
    if (ctx->cfg.precision == PDG_PRECISION_F64)
        k_check_insert<QM, double><<<grid_for(m), 256, 0, ctx->stream>>>(
            m, s, d, ctx->n, ctx->d_q, static_cast<const double *>(phi), ctx->d_free, ctx->ftop,
            ctx->d_gen, ctx->d_sum);
    else
        k_check_insert<QM, float><<<grid_for(m), 256, 0, ctx->stream>>>(
            m, s, d, ctx->n, ctx->d_q, static_cast<const float *>(phi), ctx->d_free, ctx->ftop,
            ctx->d_gen, ctx->d_sum);
}

static void launch_check_insert(pdg_ctx *ctx, int64_t m, const int32_t *s, const int32_t *d,
                                const void *phi)
{
    switch (ctx->QM) {
    case 2: check_insert_q<2>(ctx, m, s, d, phi); break;
    case 3: check_insert_q<3>(ctx, m, s, d, phi); break;
    case 4: check_insert_q<4>(ctx, m, s, d, phi); break;
    case 5: check_insert_q<5>(ctx, m, s, d, phi); break;
    case 6: check_insert_q<6>(ctx, m, s, d, phi); break;
    case 7: check_insert_q<7>(ctx, m, s, d, phi); break;
    default: check_insert_q<8>(ctx, m, s, d, phi); break;
    }
}

// ---------------------------------------------------------------- edge store
static int64_t a256(int64_t bytes) { return (bytes + 255) / 256 * 256; }

// Consecutive 256-byte aligned pieces of one scratch buffer.
struct Carve {
    char *p;
    template <typename T>
    T *take(int64_t count)
    {
        T *r = reinterpret_cast<T *>(p);
        p += a256(std::max<int64_t>(count, 1) * (int64_t)sizeof(T));
        return r;
    }
    template <typename T>
    static int64_t size(int64_t count)
    {
        return a256(std::max<int64_t>(count, 1) * (int64_t)sizeof(T));
    }
};

static pdg_status read_sum(pdg_ctx *ctx, EditSummary *h)
{
    PDG_HIP(ctx, hipGetLastError());
    PDG_HIP(ctx, hipMemcpyAsync(h, ctx->d_sum, sizeof(EditSummary), hipMemcpyDeviceToHost,
                                ctx->stream));
    PDG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return PDG_OK;
}

static pdg_status reset_sum(pdg_ctx *ctx)
{
    k_sum_reset<<<1, 64, 0, ctx->stream>>>(ctx->d_sum);
    PDG_HIP(ctx, hipGetLastError());
    return PDG_OK;
}

// Bits of a node id (radix sort keys).
static int key_bits(int64_t n)
{
    int b = 1;
    while (b < 32 && (1ll << b) < n) ++b;
    return b;
}

// Temporary storage of the library primitives used by the edit path.
static size_t prim_bytes(int64_t m2, int64_t n)
{
    size_t a = 0, b = 0, c = 0, d = 0, e = 0, f = 0;
    const uint32_t *k = nullptr;
    uint32_t *o = nullptr;
    const uint64_t *k64 = nullptr;
    uint64_t *o64 = nullptr;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, a, k, o, k, o, (int)m2, 0, 32);
    (void)hipcub::DeviceRunLengthEncode::Encode(nullptr, b, k, o, o, o, (int)m2);
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, c, k, o, (int)m2);
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, d, k64, o64, (int)m2);
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, e, k64, o64, (int)n);
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, f, k, o, (int)n);
    size_t g = 0;
    (void)hipcub::DeviceRadixSort::SortPairsDescending(nullptr, g, k, o, k, o, (int)n, 0, 16);
    return std::max({a, b, c, d, e, f, g, (size_t)256});
}

template <int QM>
static void node_base_q(pdg_ctx *ctx, int64_t nn, const uint32_t *count, const uint32_t *dnodes)
{
    k_node_base<QM><<<grid_for(nn * 64), 256, 0, ctx->stream>>>(
        nn, count, dnodes, ctx->d_lam, ctx->d_off, ctx->d_cnt, ctx->d_pool, ctx->d_params,
        ctx->d_base);
}

// base of the listed nodes (after their incidence lists changed); with
// `count`, only the first *count of the nn listed.
static void launch_node_base(pdg_ctx *ctx, int64_t nn, const uint32_t *count,
                             const uint32_t *dnodes)
{
    if (nn == 0) return;
    switch (ctx->QM) {
    case 2: node_base_q<2>(ctx, nn, count, dnodes); break;
    case 3: node_base_q<3>(ctx, nn, count, dnodes); break;
    case 4: node_base_q<4>(ctx, nn, count, dnodes); break;
    case 5: node_base_q<5>(ctx, nn, count, dnodes); break;
    case 6: node_base_q<6>(ctx, nn, count, dnodes); break;
    case 7: node_base_q<7>(ctx, nn, count, dnodes); break;
    default: node_base_q<8>(ctx, nn, count, dnodes); break;
    }
}

// Lay every segment out again in fresh buffers, with room for the batch's
// appends (runlen of the distinct nodes uniq), and free the old buffers.
// ncap / noff: scratch of n entries.
static pdg_status full_relayout(pdg_ctx *ctx, int64_t runs, const uint32_t *uniq,
                                const uint32_t *runlen, uint64_t *ncap, uint64_t *noff, void *tmp,
                                size_t tb)
{
    const int64_t n = ctx->n;
    const hipStream_t st = ctx->stream;
    k_scatter_runs<<<grid_for(runs), 256, 0, st>>>(runs, &ctx->d_sum->runs, uniq, runlen,
                                                   ctx->d_mark);
    k_full_cap<<<grid_for(n), 256, 0, st>>>(n, ctx->d_nlive, ctx->d_mark, ncap);
    PDG_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(tmp, tb, ncap, noff, (int)n, st));
    k_scan_total<<<1, 64, 0, st>>>(n, ncap, noff, &ctx->d_sum->total);
    k_unmark<<<grid_for(runs), 256, 0, st>>>(runs, &ctx->d_sum->runs, uniq, ctx->d_mark);
    EditSummary h;
    PDG_TRY(read_sum(ctx, &h));
    const uint64_t total = h.total, size = total + total / 4 + 1024;
    if (size >= 0xFFFFFFF0ull) return fail(ctx, PDG_ECAPACITY, "incidence pool exceeds 2^32 entries");
    const int64_t cap = (int64_t)size;
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
    k_fill_u32<<<grid_for(cap), 256, 0, st>>>(npool, cap, kTomb);
    PDG_HIP(ctx, hipMemsetAsync(nrp, 0, cap * ctx->RP * 8 + 256, st));
    PDG_HIP(ctx, hipMemsetAsync(nrz, 0, cap * ctx->ZW * 4 + 256, st));
    k_relocate<<<grid_for(n * 64), 256, 0, st>>>(
        n, nullptr, nullptr, ncap, noff, 0, 1, ctx->d_off, ctx->d_cnt, ctx->d_cap, ctx->d_pool,
        npool, ctx->d_ipos, ctx->d_rec_p, nrp, ctx->RP, ctx->d_rec_z, nrz, ctx->ZW);
    PDG_HIP(ctx, hipGetLastError());
    PDG_HIP(ctx, hipStreamSynchronize(st));
    if (ctx->d_pool) PDG_HIP(ctx, hipFree(ctx->d_pool));
    if (ctx->d_rec_p) PDG_HIP(ctx, hipFree(ctx->d_rec_p));
    if (ctx->d_rec_z) PDG_HIP(ctx, hipFree(ctx->d_rec_z));
    ctx->d_pool = npool;
    ctx->d_rec_p = nrp;
    ctx->d_rec_z = nrz;
    ctx->dev_pool_cap = cap;
    ctx->pool_top = (int64_t)total;
    return PDG_OK;
}

// Hub list and piece table from the segment counts, in node order.  Hubs
// are split only while a hub piece kernel's LDS chunk holds at least the
// records of one step (one record per lane group).  flag / pieces / hidx /
// pidx: scratch of n entries.
static pdg_status rebuild_hub_table(pdg_ctx *ctx, uint32_t *flag, uint32_t *pieces, uint32_t *hidx,
                                    uint32_t *pidx, void *tmp, size_t tb)
{
    ctx->hub_thr = 0;
    ctx->nh = ctx->np = 0;
    const int64_t D = ctx->D, RP = ctx->RP;
    const int64_t zr = ctx->LPI == 64 ? 2 * D * ctx->CB : D;
    const int64_t zb = (8 * D + 15) / 16 * 16;
    const int64_t K = zc_layout(ctx->QM, ctx->C) ? kZChunk : (4096 - zb - 48) / (RP * 8 + 4 * zr);
    if (K < (ctx->LPI == 64 ? 1 : 64 / ctx->LPI) || ctx->tune_hub_thr == 0) return PDG_OK;
    const int64_t n = ctx->n;
    const hipStream_t st = ctx->stream;
    k_hub_count<<<grid_for(n), 256, 0, st>>>(n, ctx->d_cnt, ctx->tune_hub_thr, ctx->tune_piece, flag,
                                             pieces);
    PDG_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(tmp, tb, flag, hidx, (int)n, st));
    PDG_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(tmp, tb, pieces, pidx, (int)n, st));
    k_scan_total<<<1, 64, 0, st>>>(n, flag, hidx, &ctx->d_sum->nh);
    k_scan_total<<<1, 64, 0, st>>>(n, pieces, pidx, &ctx->d_sum->np);
    EditSummary h;
    PDG_TRY(read_sum(ctx, &h));
    const int64_t nh = h.nh, np = h.np;
    if (nh == 0) return PDG_OK;
    // both grow with half again as much room, so that a hub list that
    // changes a little from one edit batch to the next does not reallocate
    // (a free waits for the device)
    const int64_t words = nh + (nh + 1) + 3 * np;
    if (words > ctx->hub_cap) {
        if (ctx->d_hub) PDG_HIP(ctx, hipFree(ctx->d_hub));
        ctx->d_hub = nullptr;
        ctx->hub_cap = 0;
        const int64_t cap = words + words / 2 + 256;
        PDG_TRY(dalloc(ctx, (void **)&ctx->d_hub, cap * 4));
        ctx->hub_cap = cap;
    }
    const int64_t pd = np * ctx->CB * (ctx->QM - 1) * 64;
    if (pd > ctx->part_cap) {
        if (ctx->d_part) PDG_HIP(ctx, hipFree(ctx->d_part));
        ctx->d_part = nullptr;
        ctx->part_cap = 0;
        const int64_t cap = pd + pd / 2 + 4096;
        PDG_TRY(dalloc(ctx, (void **)&ctx->d_part, cap * 8));
        ctx->part_cap = cap;
    }
    k_hub_fill<<<grid_for(n), 256, 0, st>>>(n, ctx->d_cnt, ctx->tune_piece, flag, hidx, pidx,
                                            (uint32_t)nh, (uint32_t)np, ctx->d_hub);
    PDG_HIP(ctx, hipGetLastError());
    ctx->nh = nh;
    ctx->np = np;
    ctx->hub_thr = ctx->tune_hub_thr;
    return PDG_OK;
}

// The hub table, then (chain-major primal) the node order: non-hub nodes by
// record count, largest first, ties in id order, hubs last.  Scratch as for
// rebuild_hub_table (tmp also holds a radix sort of n pairs).
static pdg_status rebuild_hubs(pdg_ctx *ctx, uint32_t *flag, uint32_t *pieces, uint32_t *hidx,
                               uint32_t *pidx, void *tmp, size_t tb)
{
    PDG_TRY(rebuild_hub_table(ctx, flag, pieces, hidx, pidx, tmp, tb));
    if (!zc_layout(ctx->QM, ctx->C)) return PDG_OK;
    const int64_t n = ctx->n;
    const hipStream_t st = ctx->stream;
    ctx->order_set = false;
    k_order_keys<<<grid_for(n), 256, 0, st>>>(n, ctx->d_cnt, ctx->hub_thr, flag, hidx);
    PDG_HIP(ctx, hipGetLastError());
    PDG_HIP(ctx, hipcub::DeviceRadixSort::SortPairsDescending(tmp, tb, flag, pieces, hidx,
                                                              ctx->d_order, (int)n, 0, 16, st));
    ctx->order_set = true;
    return PDG_OK;
}

// rebuild_hubs with scratch of its own (tuning, explicit settings)
static pdg_status rebuild_hubs_alone(pdg_ctx *ctx)
{
    const int64_t n = ctx->n;
    const size_t tb = prim_bytes(2, n);
    void *sp;
    PDG_TRY(ctx_scratch(ctx, 4 * Carve::size<uint32_t>(n) + a256((int64_t)tb), &sp));
    Carve cv{static_cast<char *>(sp)};
    uint32_t *flag = cv.take<uint32_t>(n), *pieces = cv.take<uint32_t>(n);
    uint32_t *hidx = cv.take<uint32_t>(n), *pidx = cv.take<uint32_t>(n);
    void *tmp = cv.take<char>((int64_t)tb);
    return rebuild_hubs(ctx, flag, pieces, hidx, pidx, tmp, tb);
}

struct NonZeroU64 {
    __host__ __device__ bool operator()(const uint64_t &v) const { return v != 0; }
};

template <int QM>
static void logv_q(pdg_ctx *ctx, const Graph &g, int64_t bn, int64_t be, double *pn, double *pe)
{
    const hipStream_t st = ctx->stream;
    if (g.C > 32)
        k_logv_nodes<QM, true><<<dim3((unsigned)bn, (unsigned)g.CB), 256, 0, st>>>(g, pn);
    else
        k_logv_nodes<QM, false><<<dim3((unsigned)bn, (unsigned)g.CB), 256, 0, st>>>(g, pn);
    if (be == 0) return;
    if (ctx->cfg.precision == PDG_PRECISION_F64)
        k_logv_edges<QM, double><<<dim3((unsigned)be, (unsigned)g.CB), 256, 0, st>>>(
            g, static_cast<const double *>(ctx->d_lphi), pe);
    else
        k_logv_edges<QM, float><<<dim3((unsigned)be, (unsigned)g.CB), 256, 0, st>>>(
            g, static_cast<const float *>(ctx->d_lphi), pe);
}

static void free_all(pdg_ctx *ctx)
{
    void *ps[] = {ctx->d_q,     ctx->d_lam,   ctx->d_x,     ctx->d_counts, ctx->d_src,
                  ctx->d_dst,   ctx->d_uid,   ctx->d_sq,    ctx->d_params, ctx->d_ipos,
                  ctx->d_off,   ctx->d_cnt,   ctx->d_pool,  ctx->d_rec_p,  ctx->d_rec_z,
                  ctx->d_flag,  ctx->d_scratch, ctx->d_base, ctx->d_hub, ctx->d_part,
                  ctx->d_free,  ctx->d_gen,   ctx->d_claim, ctx->d_cap,    ctx->d_nlive,
                  ctx->d_mark,  ctx->d_sum,   ctx->d_lphi,  ctx->d_dparams, ctx->d_order};
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
    if (device >= 256) return bail(fail(ctx, PDG_EINVAL, "device index above 255"));
    {
        std::lock_guard<std::mutex> lock(g_static_mu);
        if (!g_static_addr[device]) {
            void *p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
                return bail(fail(ctx, PDG_EHIP, "hipGetSymbolAddress of the static workspace failed"));
            g_static_addr[device] = p;
        }
        ctx->d_static = g_static_addr[device];
    }
    const int64_t N = cfg->node_capacity, S = cfg->edge_capacity;
    const int64_t N4 = (N + 3) / 4 * 4;  // segment tables are read per node quad
    // slot arrays are read in groups of up to kMaxDualEdgesPerWave slots
    const int64_t SP = (S + kMaxDualEdgesPerWave - 1) / kMaxDualEdgesPerWave * kMaxDualEdgesPerWave;
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
        (s = dalloc(ctx, (void **)&ctx->d_dparams, SP * thr_bytes(ctx->QM))) ||
        (s = dalloc(ctx, &ctx->d_lphi,
                    SP * ctx->QM * ctx->QM * (cfg->precision == PDG_PRECISION_F64 ? 8 : 4))) ||
        (s = dalloc(ctx, (void **)&ctx->d_ipos, SP * 8)) ||
        (s = dalloc(ctx, (void **)&ctx->d_off, N4 * 4)) ||
        (s = dalloc(ctx, (void **)&ctx->d_cnt, N4 * 4)) ||
        (s = dalloc(ctx, (void **)&ctx->d_flag, 64)) ||
        (s = dalloc(ctx, (void **)&ctx->d_free, SP * 4)) ||
        (s = dalloc(ctx, (void **)&ctx->d_gen, SP * 4)) ||
        (s = dalloc(ctx, (void **)&ctx->d_claim, SP * 4)) ||
        (s = dalloc(ctx, (void **)&ctx->d_cap, N4 * 4)) ||
        (s = dalloc(ctx, (void **)&ctx->d_nlive, N4 * 4)) ||
        (s = dalloc(ctx, (void **)&ctx->d_mark, N4 * 4)) ||
        (s = dalloc(ctx, (void **)&ctx->d_order, N4 * 4)) ||
        (s = dalloc(ctx, (void **)&ctx->d_sum, sizeof(EditSummary))))
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
        hipMemsetAsync(ctx->d_gen, 0, SP * 4, ctx->stream) != hipSuccess ||
        hipMemsetAsync(ctx->d_cap, 0, N4 * 4, ctx->stream) != hipSuccess ||
        hipMemsetAsync(ctx->d_nlive, 0, N4 * 4, ctx->stream) != hipSuccess ||
        hipMemsetAsync(ctx->d_mark, 0, N4 * 4, ctx->stream) != hipSuccess ||
        hipMemsetAsync(ctx->d_sum, 0, sizeof(EditSummary), ctx->stream) != hipSuccess)
        return bail(fail(ctx, PDG_EHIP, "initial clear failed"));
    k_store_init<<<grid_for(S), 256, 0, ctx->stream>>>(S, ctx->d_free, ctx->d_claim);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(ctx->stream) != hipSuccess)
        return bail(fail(ctx, PDG_EHIP, "store initialisation failed"));
    ctx->S = S;
    ctx->ftop = S;
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
    if (m > ctx->ftop) return fail(ctx, PDG_ECAPACITY, "edge capacity exhausted");
    if (m > (1ll << 29)) return fail(ctx, PDG_EINVAL, "more than 2^29 edges in one batch");
    PDG_TRY(set_dev(ctx));
    const hipStream_t st = ctx->stream;
    const int64_t n = ctx->n, m2 = 2 * m, mn = std::max(m2, n);
    EditSummary *sum = ctx->d_sum;
    const size_t tb = prim_bytes(m2, n);
    const int64_t bytes = 7 * Carve::size<uint32_t>(m2) + 2 * Carve::size<uint64_t>(mn) +
                          3 * Carve::size<int32_t>(m) + 4 * Carve::size<uint32_t>(n) +
                          a256((int64_t)tb);
    void *sp;
    PDG_TRY(ctx_scratch(ctx, bytes, &sp));
    Carve cv{static_cast<char *>(sp)};
    uint32_t *keys = cv.take<uint32_t>(m2), *vals = cv.take<uint32_t>(m2);
    uint32_t *keys2 = cv.take<uint32_t>(m2), *vals2 = cv.take<uint32_t>(m2);
    uint32_t *uniq = cv.take<uint32_t>(m2), *runlen = cv.take<uint32_t>(m2);
    uint32_t *runoff = cv.take<uint32_t>(m2);
    uint64_t *ncap = cv.take<uint64_t>(mn), *noff = cv.take<uint64_t>(mn);
    int32_t *dslot = cv.take<int32_t>(m), *dqs = cv.take<int32_t>(m), *dqd = cv.take<int32_t>(m);
    uint32_t *hflag = cv.take<uint32_t>(n), *hpieces = cv.take<uint32_t>(n);
    uint32_t *hidx = cv.take<uint32_t>(n), *pidx = cv.take<uint32_t>(n);
    void *tmp = cv.take<char>((int64_t)tb);

    // 1. everything checked before anything changes
    PDG_TRY(reset_sum(ctx));
    launch_check_insert(ctx, m, d_src, d_dst, d_log_phi);
    EditSummary h;
    PDG_TRY(read_sum(ctx, &h));
    if (h.flags & 1u) return fail(ctx, PDG_EINVAL, "edge endpoint out of range");
    if (h.flags & 2u) return fail(ctx, PDG_EINVAL, "self-loop is not a pairwise factor");
    if (h.flags & 4u) return fail(ctx, PDG_ECAPACITY, "uid space of a slot exhausted");
    if (h.flags & 8u) return fail(ctx, PDG_ENONPOS, "non-finite log factor entry");

    // 2. the batch's incidence entries grouped by node, batch order inside a
    //    node (stable sort); the capacity the full segments need
    k_insert_entries<<<grid_for(m2), 256, 0, st>>>(m, d_src, d_dst, ctx->d_free, ctx->ftop, keys,
                                                   vals);
    {
        size_t t2 = tb;
        PDG_HIP(ctx, hipcub::DeviceRadixSort::SortPairs(tmp, t2, keys, keys2, vals, vals2, (int)m2,
                                                        0, key_bits(n), st));
        t2 = tb;
        PDG_HIP(ctx, hipcub::DeviceRunLengthEncode::Encode(tmp, t2, keys2, uniq, runlen,
                                                           &sum->runs, (int)m2, st));
        t2 = tb;
        PDG_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(tmp, t2, runlen, runoff, (int)m2, st));
    }
    k_room<<<grid_for(m2), 256, 0, st>>>(m2, &sum->runs, uniq, runlen, ctx->d_cnt, ctx->d_cap,
                                         ctx->d_nlive, ncap);
    {
        size_t t2 = tb;
        PDG_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(tmp, t2, ncap, noff, (int)m2, st));
    }
    k_scan_total<<<1, 64, 0, st>>>(m2, ncap, noff, &sum->room);
    PDG_TRY(read_sum(ctx, &h));
    const int64_t runs = h.runs;

    // 3. room: move the full segments to the end of the pool, or lay every
    //    segment out again when the pool is too small.  From here on a failure
    //    leaves the store half changed: the context refuses every later call.
    ctx->broken = true;
    if ((uint64_t)ctx->pool_top + h.room > (uint64_t)ctx->dev_pool_cap) {
        PDG_TRY(full_relayout(ctx, runs, uniq, runlen, ncap, noff, tmp, tb));
    } else if (h.room) {
        k_relocate<<<grid_for(runs * 64), 256, 0, st>>>(
            runs, nullptr, uniq, ncap, noff, (uint64_t)ctx->pool_top, 0, ctx->d_off, ctx->d_cnt,
            ctx->d_cap, ctx->d_pool, ctx->d_pool, ctx->d_ipos, ctx->d_rec_p, ctx->d_rec_p,
            ctx->RP, ctx->d_rec_z, ctx->d_rec_z, ctx->ZW);
        PDG_HIP(ctx, hipGetLastError());
        ctx->pool_top += (int64_t)h.room;
    }

    // 4. slots and uids, appends, decomposition, records, base
    k_slot_write<<<grid_for(m), 256, 0, st>>>(m, ctx->d_free, ctx->ftop, d_src, d_dst, ctx->d_q,
                                              ctx->d_gen, ctx->d_src, ctx->d_dst, ctx->d_uid,
                                              ctx->d_sq, dslot, dqs, dqd, d_uid_out, sum);
    k_append_first<<<grid_for(runs), 256, 0, st>>>(runs, &sum->runs, uniq, runoff, ctx->d_mark);
    k_append_entries<<<grid_for(m2), 256, 0, st>>>(m2, keys2, vals2, ctx->d_mark, ctx->d_off,
                                                   ctx->d_cnt, ctx->d_pool, ctx->d_ipos);
    k_append_heads<<<grid_for(runs), 256, 0, st>>>(runs, &sum->runs, uniq, runlen, ctx->d_cnt,
                                                   ctx->d_nlive, ctx->d_mark);
    PDG_HIP(ctx, hipGetLastError());
    ctx->ftop -= m;
    ctx->live += m;
    PDG_TRY(clear_flag(ctx));
    launch_decompose(ctx->QM, ctx->cfg.precision == PDG_PRECISION_F64, m, dqs, dqd, d_log_phi,
                     dslot, ctx->d_params, ctx->d_flag, st);
    {
        const int32_t words = (int32_t)(thr_bytes(ctx->QM) / 4);
        k_copy_dual_params<<<grid_for(m * words), 256, 0, st>>>(m, words, ctx->bbytes, dslot,
                                                                ctx->d_params, ctx->d_dparams);
    }
    k_write_records<<<grid_for(m * ctx->RP), 256, 0, st>>>(m, ctx->QM, dslot, ctx->d_sq,
                                                           ctx->d_params, ctx->d_ipos,
                                                           ctx->d_rec_p);
    {
        const int32_t QQ = ctx->QM * ctx->QM;
        if (ctx->cfg.precision == PDG_PRECISION_F64)
            k_copy_tables<double><<<grid_for(m * QQ), 256, 0, st>>>(
                m, QQ, dslot, static_cast<const double *>(d_log_phi),
                static_cast<double *>(ctx->d_lphi));
        else
            k_copy_tables<float><<<grid_for(m * QQ), 256, 0, st>>>(
                m, QQ, dslot, static_cast<const float *>(d_log_phi),
                static_cast<float *>(ctx->d_lphi));
    }
    launch_node_base(ctx, runs, nullptr, uniq);
    PDG_HIP(ctx, hipGetLastError());
    PDG_TRY(rebuild_hubs(ctx, hflag, hpieces, hidx, pidx, tmp, tb));
    PDG_TRY(read_sum(ctx, &h));
    ctx->hwm = h.hwm;
    ctx->broken = false;
    ctx->gen++;
    return PDG_OK;
}

pdg_status pdg_remove_edges(pdg_ctx *ctx, int64_t m, const uint64_t *d_uid)
{
    if (!ctx) return fail(nullptr, PDG_EINVAL, "null context");
    if (ctx->phase != 0) return fail(ctx, PDG_ESTATE, "edits only between sweeps");
    if (m < 0) return fail(ctx, PDG_EINVAL, "m < 0");
    if (m == 0) return PDG_OK;
    if (!d_uid) return fail(ctx, PDG_EINVAL, "null pointer");
    if (m > (1ll << 30)) return fail(ctx, PDG_EINVAL, "more than 2^30 edges in one batch");
    PDG_TRY(set_dev(ctx));
    const hipStream_t st = ctx->stream;
    EditSummary *sum = ctx->d_sum;
    void *sp;
    PDG_TRY(ctx_scratch(ctx, Carve::size<uint32_t>(2 * m), &sp));
    uint32_t *list = static_cast<uint32_t *>(sp);

    // every uid live and named once, else nothing changes
    PDG_TRY(reset_sum(ctx));
    k_check_remove<<<grid_for(m), 256, 0, st>>>(m, d_uid, ctx->S, ctx->d_uid, ctx->d_claim, sum);
    k_check_remove2<<<grid_for(m), 256, 0, st>>>(m, d_uid, ctx->S, ctx->d_uid, ctx->d_claim, sum);
    k_claim_reset<<<grid_for(m), 256, 0, st>>>(m, d_uid, ctx->S, ctx->d_uid, ctx->d_claim);
    EditSummary h;
    PDG_TRY(read_sum(ctx, &h));
    if (h.bad != 0xFFFFFFFFu) {
        uint64_t u = 0;
        PDG_HIP(ctx, hipMemcpyAsync(&u, d_uid + h.bad, 8, hipMemcpyDeviceToHost, st));
        PDG_HIP(ctx, hipStreamSynchronize(st));
        return fail(ctx, PDG_ENOTFOUND,
                    "uid " + std::to_string(u) + " is not a live edge or is repeated in the batch");
    }
    ctx->broken = true;  // as in pdg_insert_edges: a failure from here on is fatal
    k_clear_edge_records<<<grid_for(2 * m * ctx->RP), 256, 0, st>>>(m, ctx->RP, d_uid, ctx->d_ipos,
                                                                    ctx->d_rec_p);
    k_remove_apply<<<grid_for(m), 256, 0, st>>>(m, d_uid, ctx->d_src, ctx->d_dst, ctx->d_ipos,
                                                ctx->d_pool, ctx->d_nlive, ctx->d_uid,
                                                ctx->d_free, ctx->ftop, ctx->d_mark, list, sum);
    launch_node_base(ctx, 2 * m, &sum->nlist, list);
    k_unmark<<<grid_for(2 * m), 256, 0, st>>>(2 * m, &sum->nlist, list, ctx->d_mark);
    PDG_HIP(ctx, hipGetLastError());
    ctx->ftop += m;
    ctx->live -= m;
    PDG_HIP(ctx, hipStreamSynchronize(st));
    ctx->broken = false;
    ctx->gen++;
    return PDG_OK;
}

pdg_status pdg_num_edges(pdg_ctx *ctx, int64_t *h_live)
{
    if (!ctx || !h_live) return fail(ctx, PDG_EINVAL, "null argument");
    *h_live = ctx->live;
    return PDG_OK;
}

pdg_status pdg_live_uids(pdg_ctx *ctx, uint64_t *d_uid_out)
{
    if (!ctx || !d_uid_out) return fail(ctx, PDG_EINVAL, "null argument");
    if (ctx->live == 0) return PDG_OK;
    PDG_TRY(set_dev(ctx));
    size_t tb = 0;
    PDG_HIP(ctx, hipcub::DeviceSelect::If(nullptr, tb, ctx->d_uid, d_uid_out, &ctx->d_sum->sel,
                                          (int)ctx->hwm, NonZeroU64(), ctx->stream));
    void *sp;
    PDG_TRY(ctx_scratch(ctx, (int64_t)tb + 256, &sp));
    PDG_HIP(ctx, hipcub::DeviceSelect::If(sp, tb, ctx->d_uid, d_uid_out, &ctx->d_sum->sel,
                                          (int)ctx->hwm, NonZeroU64(), ctx->stream));
    PDG_HIP(ctx, hipStreamSynchronize(ctx->stream));
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
    // every state in range before anything is copied
    PDG_TRY(clear_flag(ctx));
    const int64_t nc = ctx->n * ctx->C;
    k_check_state<<<grid_for(nc), 256, 0, ctx->stream>>>(ctx->n, ctx->C, ctx->d_q, d_x, ctx->d_flag);
    PDG_HIP(ctx, hipGetLastError());
    uint32_t bad = 0;
    PDG_TRY(read_flag(ctx, &bad));
    if (bad) return fail(ctx, PDG_EINVAL, "a state x_i >= q_i");
    PDG_HIP(ctx, hipMemcpyAsync(ctx->d_x, d_x, nc, hipMemcpyDeviceToDevice, ctx->stream));
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
    if (ctx->hwm > 0) {
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
    int64_t dw = 0, pw = 0;
    if (n_sweeps > 1 && ctx->nodes_set && ctx->phase == 0 && ctx->hwm > 0 &&
        small_waves(ctx, &dw, &pw)) {
        // small graph: batches of sweeps in one launch each (same draws)
        PDG_TRY(set_dev(ctx));
        while (n_sweeps > 0) {
            const int32_t k = (int32_t)std::min<int64_t>(n_sweeps, kSmallSweepsPerLaunch);
            if (ctx->t + k >= 0xFFFFFFFFll) return fail(ctx, PDG_ECAPACITY, "sweep counter exhausted");
            const int64_t first = std::max<int64_t>(ctx->t + 1, ctx->cfg.burn_in + 1);
            const int64_t counted = std::max<int64_t>(0, ctx->t + k - first + 1);
            if (counted && (uint64_t)(ctx->counted + counted) * (uint64_t)ctx->C > 0xFFFFFFFFull)
                return fail(ctx, PDG_ECAPACITY,
                            "marginal counters would overflow; read and reset them");
            launch_sweeps(ctx, (uint32_t)ctx->t, k, dw, pw);
            PDG_HIP(ctx, hipGetLastError());
            ctx->t += k;
            ctx->counted += counted;
            n_sweeps -= k;
        }
        return PDG_OK;
    }
    for (int64_t k = 0; k < n_sweeps; ++k) {
        PDG_TRY(pdg_dual_phase(ctx));
        PDG_TRY(pdg_primal_phase(ctx));
    }
    return PDG_OK;
}

struct pdg_graph {
    std::vector<pdg_ctx *> ctxs;
    std::vector<uint64_t> gens;
    int32_t n_sweeps = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

pdg_status pdg_graph_create(pdg_ctx *const *ctxs, int32_t n_ctx, int32_t n_sweeps, pdg_graph **out)
{
    if (!ctxs || !out || n_ctx < 1) return fail(nullptr, PDG_EINVAL, "bad argument");
    *out = nullptr;
    if (n_sweeps < 1 || n_sweeps > 4096) return fail(nullptr, PDG_EINVAL, "n_sweeps must be in [1, 4096]");
    for (int32_t i = 0; i < n_ctx; ++i) {
        pdg_ctx *c = ctxs[i];
        if (!c) return fail(nullptr, PDG_EINVAL, "null context");
        if (!c->nodes_set) return fail(nullptr, PDG_ESTATE, "pdg_set_nodes first");
        if (c->phase != 0) return fail(nullptr, PDG_ESTATE, "capture between sweeps");
        if (c->device != ctxs[0]->device || c->stream != ctxs[0]->stream)
            return fail(nullptr, PDG_EINVAL, "every context of a graph needs the same device and stream");
        for (int32_t j = 0; j < i; ++j)
            if (ctxs[j] == c) return fail(nullptr, PDG_EINVAL, "a context appears twice");
    }
    if (ctxs[0]->broken || hipSetDevice(ctxs[0]->device) != hipSuccess)
        return fail(nullptr, PDG_ESTATE, "context unusable");
    pdg_graph *gr = new (std::nothrow) pdg_graph();
    if (!gr) return fail(nullptr, PDG_ENOMEM, "host allocation failed");
    gr->ctxs.assign(ctxs, ctxs + n_ctx);
    for (pdg_ctx *c : gr->ctxs) gr->gens.push_back(c->gen);
    gr->n_sweeps = n_sweeps;
    // capture on a stream of our own (the contexts' stream may be the legacy
    // default stream, which cannot be captured); replays go to theirs
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
        delete gr;
        return fail(nullptr, PDG_EHIP, "hipStreamCreateWithFlags failed");
    }
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    std::vector<hipStream_t> saved;
    for (pdg_ctx *c : gr->ctxs) {
        saved.push_back(c->stream);
        c->stream = cs;
        c->replay = true;
    }
    if (e == hipSuccess) {
        for (int32_t k = 0; k < n_sweeps && e == hipSuccess; ++k)
            for (pdg_ctx *c : gr->ctxs) {
                k_tick<<<1, 64, 0, cs>>>(c->d_flag + 8);
                launch_dual(c, 0u);
                launch_primal(c, 0u, 0);
                e = hipGetLastError();
                if (e != hipSuccess) break;
            }
        hipGraph_t graph = nullptr;
        const hipError_t e2 = hipStreamEndCapture(cs, &graph);
        if (e == hipSuccess) e = e2;
        gr->graph = graph;
    }
    for (size_t i = 0; i < gr->ctxs.size(); ++i) {
        gr->ctxs[i]->stream = saved[i];
        gr->ctxs[i]->replay = false;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&gr->exec, gr->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
        if (gr->graph) (void)hipGraphDestroy(gr->graph);
        delete gr;
        return fail(nullptr, PDG_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    }
    *out = gr;
    return PDG_OK;
}

pdg_status pdg_graph_launch(pdg_graph *gr)
{
    if (!gr) return fail(nullptr, PDG_EINVAL, "null graph");
    const int64_t n = gr->n_sweeps;
    for (size_t i = 0; i < gr->ctxs.size(); ++i) {
        pdg_ctx *c = gr->ctxs[i];
        if (c->gen != gr->gens[i])
            return fail(nullptr, PDG_ESTATE, "the edges changed since the sweeps were captured; capture again");
        if (c->phase != 0) return fail(nullptr, PDG_ESTATE, "replay between sweeps");
        if (c->t + n >= 0xFFFFFFFFll) return fail(nullptr, PDG_ECAPACITY, "sweep counter exhausted");
        const int64_t first = std::max<int64_t>(c->t + 1, c->cfg.burn_in + 1);
        const int64_t counted = std::max<int64_t>(0, c->t + n - first + 1);
        if (counted && (uint64_t)(c->counted + counted) * (uint64_t)c->C > 0xFFFFFFFFull)
            return fail(nullptr, PDG_ECAPACITY, "marginal counters would overflow; read and reset them");
    }
    pdg_ctx *c0 = gr->ctxs[0];
    for (pdg_ctx *c : gr->ctxs)
        if (c->broken) return fail(nullptr, PDG_ESTATE, "a context of the graph is unusable");
    PDG_HIP(nullptr, hipSetDevice(c0->device));
    for (pdg_ctx *c : gr->ctxs)
        k_set_counter<<<1, 64, 0, c0->stream>>>(c->d_flag + 8, (uint32_t)c->t);
    PDG_HIP(nullptr, hipGetLastError());
    PDG_HIP(nullptr, hipGraphLaunch(gr->exec, c0->stream));
    for (pdg_ctx *c : gr->ctxs) {
        const int64_t first = std::max<int64_t>(c->t + 1, c->cfg.burn_in + 1);
        c->counted += std::max<int64_t>(0, c->t + n - first + 1);
        c->t += n;
    }
    return PDG_OK;
}

pdg_status pdg_graph_destroy(pdg_graph *gr)
{
    if (!gr) return PDG_OK;
    if (!gr->ctxs.empty()) (void)hipSetDevice(gr->ctxs[0]->device);
    if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
    if (gr->graph) (void)hipGraphDestroy(gr->graph);
    delete gr;
    return PDG_OK;
}

static void tuning_of(const pdg_ctx *ctx, pdg_tuning *o)
{
    o->dual_edges_per_wave = ctx->tune_e64;
    o->binary_groups_per_wave = ctx->tune_ebin;
    o->hub_threshold = (int32_t)ctx->tune_hub_thr;
    o->hub_piece = (int32_t)ctx->tune_piece;
}

static bool tuning_valid(const pdg_tuning *t)
{
    auto e_ok = [](int32_t e) { return e == 2 || e == 4 || e == 8; };
    return e_ok(t->dual_edges_per_wave) && e_ok(t->binary_groups_per_wave) &&
           (t->hub_threshold == 0 || (t->hub_threshold >= 32 && t->hub_threshold <= (1 << 20))) &&
           t->hub_piece >= 16 && t->hub_piece <= 4096;
}

pdg_status pdg_get_tuning(pdg_ctx *ctx, pdg_tuning *h_out)
{
    if (!ctx || !h_out) return fail(ctx, PDG_EINVAL, "null argument");
    tuning_of(ctx, h_out);
    h_out->dual_ms = h_out->primal_ms = -1.0f;
    return PDG_OK;
}

pdg_status pdg_set_tuning(pdg_ctx *ctx, const pdg_tuning *h_in)
{
    if (!ctx || !h_in) return fail(ctx, PDG_EINVAL, "null argument");
    if (!tuning_valid(h_in)) return fail(ctx, PDG_EINVAL, "tuning values out of range");
    if (ctx->phase != 0) return fail(ctx, PDG_ESTATE, "tuning between sweeps");
    PDG_TRY(set_dev(ctx));
    ctx->tune_e64 = h_in->dual_edges_per_wave;
    ctx->tune_ebin = h_in->binary_groups_per_wave;
    ctx->tune_hub_thr = (uint32_t)h_in->hub_threshold;
    ctx->tune_piece = (uint32_t)h_in->hub_piece;
    if (ctx->nodes_set) PDG_TRY(rebuild_hubs_alone(ctx));
    ctx->gen++;  // captured graphs hold the old launch shapes
    return PDG_OK;
}

pdg_status pdg_tune(pdg_ctx *ctx, int32_t reps, pdg_tuning *h_out)
{
    if (!ctx || !h_out) return fail(ctx, PDG_EINVAL, "null argument");
    if (reps < 1 || reps > 1000) return fail(ctx, PDG_EINVAL, "reps must be in [1, 1000]");
    if (!ctx->nodes_set) return fail(ctx, PDG_ESTATE, "pdg_set_nodes first");
    if (ctx->phase != 0) return fail(ctx, PDG_ESTATE, "tuning between sweeps");
    PDG_TRY(set_dev(ctx));
    const hipStream_t st = ctx->stream;
    const int64_t nc = ctx->n * ctx->C;
    uint8_t *xsave = nullptr;
    PDG_TRY(dalloc(ctx, (void **)&xsave, nc));
    hipEvent_t ea = nullptr, eb = nullptr;
    pdg_status res = PDG_OK;
    auto done = [&](pdg_status r) {
        if (ea) (void)hipEventDestroy(ea);
        if (eb) (void)hipEventDestroy(eb);
        (void)hipFree(xsave);
        return r;
    };
    if (hipEventCreate(&ea) != hipSuccess || hipEventCreate(&eb) != hipSuccess)
        return done(fail(ctx, PDG_EHIP, "hipEventCreate failed"));
    if (hipMemcpyAsync(xsave, ctx->d_x, nc, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return done(fail(ctx, PDG_EHIP, "state copy failed"));
    const uint32_t t = (uint32_t)ctx->t + 1u;
    auto time_it = [&](auto &&launch, float *ms) -> pdg_status {
        launch();
        if (hipEventRecord(ea, st) != hipSuccess) return fail(ctx, PDG_EHIP, "hipEventRecord failed");
        for (int r = 0; r < reps; ++r) launch();
        if (hipEventRecord(eb, st) != hipSuccess || hipEventSynchronize(eb) != hipSuccess ||
            hipGetLastError() != hipSuccess || hipEventElapsedTime(ms, ea, eb) != hipSuccess)
            return fail(ctx, PDG_EHIP, "timing failed");
        *ms /= (float)reps;
        return PDG_OK;
    };
    // 1. the dual's tiling: edges per wave (33 or more chains), item groups per
    //    wave (binary records with 8 or 16 chains); the draws do not depend on it
    float best_d = 0.f;
    const bool d64 = ctx->LPI == 64, dbin = ctx->QM == 2 && (ctx->LPI == 8 || ctx->LPI == 16);
    if (ctx->hwm > 0 && (d64 || dbin)) {
        int best_e = 4;
        best_d = 1e30f;
        for (int e : {2, 4, 8}) {
            (d64 ? ctx->tune_e64 : ctx->tune_ebin) = e;
            float ms = 0.f;
            res = time_it([&] { launch_dual(ctx, t); }, &ms);
            if (res != PDG_OK) return done(res);
            if (ms < best_d) { best_d = ms; best_e = e; }
        }
        (d64 ? ctx->tune_e64 : ctx->tune_ebin) = best_e;
    } else if (ctx->hwm > 0) {
        res = time_it([&] { launch_dual(ctx, t); }, &best_d);
        if (res != PDG_OK) return done(res);
    } else {
        launch_dual(ctx, t);
    }
    // 2. hubs: threshold and piece size of the split (the primal from the duals
    //    just drawn, without counting; x is restored afterwards)
    float best_p = 1e30f;
    uint32_t bt = ctx->tune_hub_thr, bp = ctx->tune_piece;
    const uint32_t thrs[] = {0u, 128u, 256u, 512u, 1024u};
    const uint32_t pieces[] = {64u, 128u, 256u};
    for (uint32_t th : thrs) {
        for (uint32_t pc : pieces) {
            if (th == 0 && pc != 128u) continue;
            ctx->tune_hub_thr = th;
            ctx->tune_piece = pc;
            res = rebuild_hubs_alone(ctx);
            if (res != PDG_OK) return done(res);
            if (th != 0 && ctx->nh == 0) continue;  // no node above this threshold
            float ms = 0.f;
            res = time_it([&] { launch_primal(ctx, t, 0); }, &ms);
            if (res != PDG_OK) return done(res);
            if (ms < best_p) { best_p = ms; bt = th; bp = pc; }
        }
    }
    ctx->tune_hub_thr = bt;
    ctx->tune_piece = bp;
    res = rebuild_hubs_alone(ctx);
    if (res != PDG_OK) return done(res);
    if (hipMemcpyAsync(ctx->d_x, xsave, nc, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return done(fail(ctx, PDG_EHIP, "state restore failed"));
    ctx->gen++;
    tuning_of(ctx, h_out);
    h_out->dual_ms = best_d;
    h_out->primal_ms = best_p;
    return done(PDG_OK);
}

pdg_status pdg_get_duals(pdg_ctx *ctx, int64_t m, const uint64_t *d_uid, uint64_t *d_theta_out)
{
    if (!ctx) return fail(nullptr, PDG_EINVAL, "null context");
    if (m < 0) return fail(ctx, PDG_EINVAL, "m < 0");
    if (m == 0) return PDG_OK;
    if (!d_uid || !d_theta_out) return fail(ctx, PDG_EINVAL, "null pointer");
    PDG_TRY(set_dev(ctx));
    void *sp;
    PDG_TRY(ctx_scratch(ctx, 4 * m + 64, &sp));
    int32_t *slots = static_cast<int32_t *>(sp);
    PDG_TRY(reset_sum(ctx));
    k_uid_slots<<<grid_for(m), 256, 0, ctx->stream>>>(m, d_uid, ctx->S, ctx->d_uid, slots,
                                                      ctx->d_sum);
    EditSummary h;
    PDG_TRY(read_sum(ctx, &h));
    if (h.bad != 0xFFFFFFFFu) return fail(ctx, PDG_ENOTFOUND, "uid is not a live edge");
    k_get_duals<<<grid_for(m * ctx->C), 256, 0, ctx->stream>>>(m, ctx->QM, make_graph(ctx), slots,
                                                               d_theta_out);
    PDG_HIP(ctx, hipGetLastError());
    PDG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return PDG_OK;
}

namespace pdg {

// Bytes of workspace one log V call needs: a row of per-chain partial sums per
// node block and edge block, the reduction's middle rows and the final row.
static int64_t log_v_bytes(const pdg_ctx *ctx, int64_t *bn, int64_t *be, int64_t *nb)
{
    *bn = cdiv(ctx->n, 16);
    *be = cdiv(ctx->hwm, 4 * kLvEdges);
    const int64_t rows = *bn + *be, row = (int64_t)ctx->CB * 64;
    *nb = std::min<int64_t>(rows, 1024);
    return (rows + *nb + 1) * row * 8;
}

// log V into d_out with the workspace `ws` (at least log_v_bytes): node and edge
// kernels write every row, the two reductions read only rows written before.
static pdg_status log_v_into(pdg_ctx *ctx, double *d_out, double *ws, int64_t bn, int64_t be,
                             int64_t nb)
{
    const Graph g = make_graph(ctx);
    const int64_t rows = bn + be, row = (int64_t)g.CB * 64, chunk = cdiv(rows, nb);
    double *pn = ws, *pe = pn + bn * row, *mid = pn + rows * row;
    switch (ctx->QM) {
    case 2: logv_q<2>(ctx, g, bn, be, pn, pe); break;
    case 3: logv_q<3>(ctx, g, bn, be, pn, pe); break;
    case 4: logv_q<4>(ctx, g, bn, be, pn, pe); break;
    case 5: logv_q<5>(ctx, g, bn, be, pn, pe); break;
    case 6: logv_q<6>(ctx, g, bn, be, pn, pe); break;
    case 7: logv_q<7>(ctx, g, bn, be, pn, pe); break;
    default: logv_q<8>(ctx, g, bn, be, pn, pe); break;
    }
    // node rows then edge rows, in row order: partial sums of nb ranges, then
    // the ranges in order
    k_logv_reduce<<<dim3((unsigned)nb, (unsigned)g.CB), 64, 0, ctx->stream>>>(rows, chunk, g.CB,
                                                                              pn, mid);
    double *fin = mid + nb * row;
    k_logv_reduce<<<dim3(1, (unsigned)g.CB), 64, 0, ctx->stream>>>(nb, nb, g.CB, mid, fin);
    PDG_HIP(ctx, hipGetLastError());
    PDG_HIP(ctx, hipMemcpyAsync(d_out, fin, (size_t)ctx->C * 8, hipMemcpyDeviceToDevice,
                                ctx->stream));
    return PDG_OK;
}

}  // namespace pdg

pdg_status pdg_log_v(pdg_ctx *ctx, double *d_out)
{
    if (!ctx || !d_out) return fail(ctx, PDG_EINVAL, "null argument");
    if (ctx->phase != 1) return fail(ctx, PDG_ESTATE, "log V is taken between the two phases");
    PDG_TRY(set_dev(ctx));
    int64_t bn, be, nb;
    const int64_t bytes = log_v_bytes(ctx, &bn, &be, &nb);
    void *sp;
    PDG_TRY(ctx_scratch(ctx, bytes + 256, &sp));
    return log_v_into(ctx, d_out, static_cast<double *>(sp), bn, be, nb);
}

pdg_status pdg_log_v_noalloc(pdg_ctx *ctx, double *d_out)
{
    if (!ctx || !d_out) return fail(ctx, PDG_EINVAL, "null argument");
    if (ctx->phase != 1) return fail(ctx, PDG_ESTATE, "log V is taken between the two phases");
    PDG_TRY(set_dev(ctx));
    int64_t bn, be, nb;
    const int64_t bytes = log_v_bytes(ctx, &bn, &be, &nb);
    if (bytes > kStaticScratchBytes)
        return fail(ctx, PDG_ECAPACITY,
                    "log V of this graph needs " + std::to_string(bytes) +
                        " bytes of workspace; the static workspace holds " +
                        std::to_string(kStaticScratchBytes));
    return log_v_into(ctx, d_out, static_cast<double *>(ctx->d_static), bn, be, nb);
}

pdg_status pdg_get_marginals(pdg_ctx *ctx, double *d_out, int64_t *h_samples)
{
    if (!ctx || !d_out) return fail(ctx, PDG_EINVAL, "null argument");
    PDG_TRY(set_dev(ctx));
    const int64_t samples = ctx->counted * ctx->C;
    const int64_t nq = ctx->n * ctx->QM;
    k_marginals<<<grid_for(nq), 256, 0, ctx->stream>>>(nq, ctx->d_counts, (double)samples, d_out);
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

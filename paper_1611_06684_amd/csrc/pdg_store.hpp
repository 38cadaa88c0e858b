// Kernels of the edge store: slot allocation, incidence segments and their
// relocation, removal, and the hub table, all decided on the device.
//
// Factors come and go between sweeps (the abstract, Sec. 1 and Sec. 6 of the
// paper motivate the method by this setting); the sampler needs no colouring,
// so an edit only has to keep, per node, the list of its incidence records.
//
// Device state besides the sweep arrays:
//   free   int32  [S]     free-slot stack; the host keeps its height ftop.
//                         Insert k of a batch takes free[ftop - 1 - k];
//                         removal k pushes its slot at free[ftop + k].
//   gen    uint32 [S]     generation of each slot; uid = gen << 32 | slot.
//   claim  uint32 [S]     all ones between calls (duplicate test of removals).
//   cap    uint32 [n]     capacity of the node's segment; cnt <= cap.
//   nlive  uint32 [n]     live (non-tombstone) entries of the segment.
//   mark   uint32 [n]     zero between calls (per-call node scratch).
//   sum    EditSummary    the few numbers the host reads back.
// Determinism: the new entries of a node are appended in batch order (a
// stable sort by node), relocation offsets come from a prefix sum in node
// order, and compaction keeps the order of live entries, so the record order
// of every node -- the summation order of its field -- depends only on the
// sequence of edit batches.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdg {

struct EditSummary {
    uint32_t flags;   // insert check: 1 endpoint out of range, 2 self-loop,
                      // 4 uid space of a slot exhausted, 8 non-finite table entry
    uint32_t bad;     // first batch index that is not a live uid or repeats one (~0: none)
    uint32_t runs;    // distinct endpoint nodes of an insert batch
    uint32_t hwm;     // slots [0, hwm) may be live
    uint32_t nlist;   // distinct endpoint nodes of a remove batch
    uint32_t nh, np;  // hubs and hub pieces
    uint32_t sel;     // items selected by a compaction
    uint64_t room;    // pool entries the batch's relocations take
    uint64_t total;   // entries of a full re-layout
};

__host__ __device__ constexpr uint32_t seg_slack(uint32_t k) { return k / 4u > 2u ? k / 4u : 2u; }

// Capacity of a segment that must hold `want` entries.
__host__ __device__ inline uint64_t seg_cap(uint64_t want)
{
    return want ? want + seg_slack((uint32_t)want) : 0;
}

__global__ void k_store_init(int64_t S, int32_t *__restrict__ free_stack,
                             uint32_t *__restrict__ claim)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= S) return;
    free_stack[j] = (int32_t)(S - 1 - j);  // slot 0 is taken first
    claim[j] = 0xFFFFFFFFu;
}

__global__ void k_sum_reset(EditSummary *sum)
{
    if (threadIdx.x == 0) {
        sum->flags = 0;
        sum->bad = 0xFFFFFFFFu;
        sum->runs = sum->nlist = sum->nh = sum->np = sum->sel = 0;
        sum->room = sum->total = 0;
    }
}

// Insert batch, before anything changes: endpoints, slot generations and
// finiteness of the used table entries.
template <int QM, typename T>
__global__ void k_check_insert(int64_t m, const int32_t *__restrict__ src,
                               const int32_t *__restrict__ dst, int64_t n,
                               const uint8_t *__restrict__ q, const T *__restrict__ phi,
                               const int32_t *__restrict__ free_stack, int64_t ftop,
                               const uint32_t *__restrict__ gen, EditSummary *sum)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const int32_t a = src[k], b = dst[k];
    uint32_t f = 0;
    if (a < 0 || a >= n || b < 0 || b >= n) {
        f = 1;
    } else if (a == b) {
        f = 2;
    } else {
        if (gen[free_stack[ftop - 1 - k]] == 0xFFFFFFFFu) f |= 4;
        const int qs = q[a], qd = q[b];
        const T *L = phi + k * QM * QM;
        for (int r = 0; r < qs; ++r)
            for (int c = 0; c < qd; ++c)
                if (!isfinite((double)L[r * QM + c])) f |= 8;
    }
    if (f) atomicOr(&sum->flags, f);
}

// Incidence entries of an insert batch in batch order: entry 2k + side has
// key = its node and value = slot << 1 | side (side 0: the node is src).
__global__ void k_insert_entries(int64_t m, const int32_t *__restrict__ src,
                                 const int32_t *__restrict__ dst,
                                 const int32_t *__restrict__ free_stack, int64_t ftop,
                                 uint32_t *__restrict__ keys, uint32_t *__restrict__ vals)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= 2 * m) return;
    const int64_t k = j >> 1;
    const uint32_t side = (uint32_t)(j & 1);
    const uint32_t slot = (uint32_t)free_stack[ftop - 1 - k];
    keys[j] = (uint32_t)(side ? dst[k] : src[k]);
    vals[j] = (slot << 1) | side;
}

// Slots of the new edges: generation, uid, endpoints, state counts.
__global__ void k_slot_write(int64_t m, const int32_t *__restrict__ free_stack, int64_t ftop,
                             const int32_t *__restrict__ src_in, const int32_t *__restrict__ dst_in,
                             const uint8_t *__restrict__ q, uint32_t *__restrict__ gen,
                             int32_t *__restrict__ src, int32_t *__restrict__ dst,
                             uint64_t *__restrict__ uid, uint8_t *__restrict__ sq,
                             int32_t *__restrict__ slots_out, int32_t *__restrict__ qs_out,
                             int32_t *__restrict__ qd_out, uint64_t *__restrict__ uid_out,
                             EditSummary *sum)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const int32_t s = free_stack[ftop - 1 - k], a = src_in[k], b = dst_in[k];
    const uint32_t g = gen[s] + 1u;
    gen[s] = g;
    const uint64_t u = ((uint64_t)g << 32) | (uint32_t)s;
    src[s] = a;
    dst[s] = b;
    uid[s] = u;
    const uint8_t qa = q[a], qb = q[b];
    sq[s] = (uint8_t)(qa | (qb << 4));
    slots_out[k] = s;
    qs_out[k] = qa;
    qd_out[k] = qb;
    if (uid_out) uid_out[k] = u;
    atomicMax(&sum->hwm, (uint32_t)s + 1u);
}

// Per distinct node u of the batch (runs of the sorted keys): the capacity
// of a new segment when the appends do not fit, else 0.
__global__ void k_room(int64_t bound, const uint32_t *__restrict__ nruns,
                       const uint32_t *__restrict__ uniq, const uint32_t *__restrict__ runlen,
                       const uint32_t *__restrict__ cnt, const uint32_t *__restrict__ cap,
                       const uint32_t *__restrict__ nlive, uint64_t *__restrict__ ncap)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= bound) return;
    if (u >= (int64_t)*nruns) {
        ncap[u] = 0;
        return;
    }
    const uint32_t i = uniq[u], k = runlen[u];
    ncap[u] = (uint64_t)cnt[i] + k > cap[i] ? seg_cap((uint64_t)nlive[i] + k) : 0;
}

// *out = v[bound - 1] + ex[bound - 1] (total of an exclusive prefix sum)
template <typename T, typename R>
__global__ void k_scan_total(int64_t bound, const T *__restrict__ v, const T *__restrict__ ex,
                             R *out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *out = (R)(bound ? v[bound - 1] + ex[bound - 1] : 0);
}

// mark[uniq[u]] = runlen[u] for the batch's distinct nodes.
__global__ void k_scatter_runs(int64_t bound, const uint32_t *__restrict__ nruns,
                               const uint32_t *__restrict__ uniq,
                               const uint32_t *__restrict__ v, uint32_t *__restrict__ mark)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < bound && u < (int64_t)*nruns) mark[uniq[u]] = v[u];
}

__global__ void k_unmark(int64_t bound, const uint32_t *__restrict__ count,
                         const uint32_t *__restrict__ nodes, uint32_t *__restrict__ mark)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < bound && u < (int64_t)*count) mark[nodes[u]] = 0;
}

// Full re-layout: new capacity of every node (live entries plus the batch's
// appends, held in mark).
__global__ void k_full_cap(int64_t n, const uint32_t *__restrict__ nlive,
                           const uint32_t *__restrict__ mark, uint64_t *__restrict__ ncap)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) ncap[i] = seg_cap((uint64_t)nlive[i] + mark[i]);
}

// Segment relocation, one wave per item.  Item u is node nodes[u] (or u when
// nodes is null).  In a partial pass only items with ncap[u] > 0 move, to
// base + noff[u] inside the same buffers (the new space lies beyond every
// segment); a full pass moves every node into fresh buffers.  The live
// entries keep their order; their records and ipos follow them; the node's
// header becomes (new offset, live count, ncap).
__global__ __launch_bounds__(256) void k_relocate(
    int64_t bound, const uint32_t *__restrict__ count, const uint32_t *__restrict__ nodes,
    const uint64_t *__restrict__ ncap, const uint64_t *__restrict__ noff, uint64_t base, int full,
    uint32_t *__restrict__ off, uint32_t *__restrict__ cnt, uint32_t *__restrict__ cap,
    const uint32_t *pool_in, uint32_t *pool_out, uint32_t *__restrict__ ipos, const double *rp_in,
    double *rp_out, int32_t RP, const uint32_t *rz_in, uint32_t *rz_out, int64_t ZW)
{
    const int64_t u = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t nn = count ? (bound < (int64_t)*count ? bound : (int64_t)*count) : bound;
    if (u >= nn) return;
    const uint64_t nc = ncap[u];
    if (!full && nc == 0) return;
    const uint32_t i = nodes ? nodes[u] : (uint32_t)u;
    const uint32_t o = off[i], c = cnt[i];
    const uint64_t no = base + noff[u];
    uint32_t wr = 0;
    for (uint32_t b = 0; b < c; b += 64) {
        const uint32_t k = b + (uint32_t)lane;
        const uint32_t e = k < c ? pool_in[o + k] : kTomb;
        const bool live = e != kTomb;
        const uint64_t mask = __ballot(live);
        if (live) {
            const uint64_t to = no + wr + __popcll(mask & ((1ull << lane) - 1ull));
            const uint64_t from = (uint64_t)o + k;
            pool_out[to] = e;
            ipos[e] = (uint32_t)to;
            for (int d = 0; d < RP; ++d) rp_out[to * RP + d] = rp_in[from * RP + d];
            for (int64_t d = 0; d < ZW; ++d) rz_out[to * ZW + d] = rz_in[from * ZW + d];
        }
        wr += (uint32_t)__popcll(mask);
    }
    if (lane == 0) {
        off[i] = (uint32_t)no;
        cnt[i] = wr;
        cap[i] = (uint32_t)nc;
    }
}

// Appends of an insert batch.  sorted keys / vals: the batch's entries
// stably sorted by node; runoff[u]: first position of run u.  Entry p of run
// u goes to position cnt + (p - runoff[u]) of its node's segment.
__global__ void k_append_first(int64_t bound, const uint32_t *__restrict__ nruns,
                               const uint32_t *__restrict__ uniq,
                               const uint32_t *__restrict__ runoff, uint32_t *__restrict__ first)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < bound && u < (int64_t)*nruns) first[uniq[u]] = runoff[u];
}

__global__ void k_append_entries(int64_t total, const uint32_t *__restrict__ keys,
                                 const uint32_t *__restrict__ vals,
                                 const uint32_t *__restrict__ first,
                                 const uint32_t *__restrict__ off, const uint32_t *__restrict__ cnt,
                                 uint32_t *__restrict__ pool, uint32_t *__restrict__ ipos)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= total) return;
    const uint32_t i = keys[p], e = vals[p];
    const uint32_t at = off[i] + cnt[i] + (uint32_t)(p - first[i]);
    pool[at] = e;
    ipos[e] = at;
}

// Headers after the appends; also clears first[] (the node scratch).
__global__ void k_append_heads(int64_t bound, const uint32_t *__restrict__ nruns,
                               const uint32_t *__restrict__ uniq,
                               const uint32_t *__restrict__ runlen, uint32_t *__restrict__ cnt,
                               uint32_t *__restrict__ nlive, uint32_t *__restrict__ first)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= bound || u >= (int64_t)*nruns) return;
    const uint32_t i = uniq[u], k = runlen[u];
    cnt[i] += k;
    nlive[i] += k;
    first[i] = 0;
}

// Remove batch, before anything changes: every uid must be live and appear
// once.  Pass 1 records, per slot, the smallest batch index naming it; pass 2
// flags any other index; pass 3 restores claim.  sum->bad = smallest bad index.
__device__ __forceinline__ bool uid_live(uint64_t u, int64_t S, const uint64_t *__restrict__ uid)
{
    const uint64_t s = u & 0xFFFFFFFFull;
    return u != 0 && (int64_t)s < S && uid[s] == u;
}

__global__ void k_check_remove(int64_t m, const uint64_t *__restrict__ uids, int64_t S,
                               const uint64_t *__restrict__ uid, uint32_t *__restrict__ claim,
                               EditSummary *sum)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const uint64_t u = uids[k];
    if (!uid_live(u, S, uid))
        atomicMin(&sum->bad, (uint32_t)k);
    else
        atomicMin(&claim[u & 0xFFFFFFFFull], (uint32_t)k);
}

__global__ void k_check_remove2(int64_t m, const uint64_t *__restrict__ uids, int64_t S,
                                const uint64_t *__restrict__ uid,
                                const uint32_t *__restrict__ claim, EditSummary *sum)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const uint64_t u = uids[k];
    if (uid_live(u, S, uid) && claim[u & 0xFFFFFFFFull] != (uint32_t)k)
        atomicMin(&sum->bad, (uint32_t)k);
}

__global__ void k_claim_reset(int64_t m, const uint64_t *__restrict__ uids, int64_t S,
                              const uint64_t *__restrict__ uid, uint32_t *__restrict__ claim)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const uint64_t u = uids[k];
    if (uid_live(u, S, uid)) claim[u & 0xFFFFFFFFull] = 0xFFFFFFFFu;
}

// Remove a validated batch: tombstone both incidence entries, free the slot
// (pushed in batch order), and list each endpoint node once (mark).
__global__ void k_remove_apply(int64_t m, const uint64_t *__restrict__ uids,
                               const int32_t *__restrict__ src, const int32_t *__restrict__ dst,
                               const uint32_t *__restrict__ ipos, uint32_t *__restrict__ pool,
                               uint32_t *__restrict__ nlive, uint64_t *__restrict__ uid,
                               int32_t *__restrict__ free_stack, int64_t ftop,
                               uint32_t *__restrict__ mark, uint32_t *__restrict__ list,
                               EditSummary *sum)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const uint32_t s = (uint32_t)(uids[k] & 0xFFFFFFFFull);
    const int32_t a = src[s], b = dst[s];
    pool[ipos[2 * (uint64_t)s]] = kTomb;
    pool[ipos[2 * (uint64_t)s + 1]] = kTomb;
    atomicSub(&nlive[a], 1u);
    atomicSub(&nlive[b], 1u);
    uid[s] = 0;
    free_stack[ftop + k] = (int32_t)s;
    if (atomicExch(&mark[a], 1u) == 0u) list[atomicAdd(&sum->nlist, 1u)] = (uint32_t)a;
    if (atomicExch(&mark[b], 1u) == 0u) list[atomicAdd(&sum->nlist, 1u)] = (uint32_t)b;
}

// Zero both records of each removed edge (a zero record adds nothing).
__global__ void k_clear_edge_records(int64_t m, int32_t RP, const uint64_t *__restrict__ uids,
                                     const uint32_t *__restrict__ ipos, double *__restrict__ rec_p)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 2 * m * RP) return;
    const int64_t ks = idx / RP;
    const int64_t j = idx - ks * RP;
    const uint64_t s = uids[ks >> 1] & 0xFFFFFFFFull;
    rec_p[(uint64_t)ipos[2 * s + (ks & 1)] * RP + j] = 0.0;
}

// uid -> slot for lookups; sum->bad = smallest index whose uid is not live.
__global__ void k_uid_slots(int64_t m, const uint64_t *__restrict__ uids, int64_t S,
                            const uint64_t *__restrict__ uid, int32_t *__restrict__ slots,
                            EditSummary *sum)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const uint64_t u = uids[k];
    const bool ok = uid_live(u, S, uid);
    slots[k] = ok ? (int32_t)(u & 0xFFFFFFFFull) : 0;
    if (!ok) atomicMin(&sum->bad, (uint32_t)k);
}

// Hub table: a node with more than thr entries is a hub, cut into pieces of
// piece entries.  flag / pieces per node, then (after prefix sums in node
// order) the table hnode[nh] | hpfirst[nh + 1] | pnode[np] | pfirst[np] | pn[np].
__global__ void k_hub_count(int64_t n, const uint32_t *__restrict__ cnt, uint32_t thr,
                            uint32_t piece, uint32_t *__restrict__ flag,
                            uint32_t *__restrict__ pieces)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t c = cnt[i];
    const bool h = c > thr;
    flag[i] = h ? 1u : 0u;
    pieces[i] = h ? (c + piece - 1) / piece : 0u;
}

// Sort keys of the node order of k_primal32z: the record count (hubs, drawn
// by the hub kernels, 0), capped at 2^16 - 1; values the node ids.
__global__ void k_order_keys(int64_t n, const uint32_t *__restrict__ cnt, uint32_t heavy,
                             uint32_t *__restrict__ keys, uint32_t *__restrict__ ids)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t c = cnt[i];
    keys[i] = heavy && c > heavy ? 0u : (c < 0xFFFFu ? c : 0xFFFFu);
    ids[i] = (uint32_t)i;
}

__global__ void k_hub_fill(int64_t n, const uint32_t *__restrict__ cnt, uint32_t piece,
                           const uint32_t *__restrict__ flag, const uint32_t *__restrict__ hidx,
                           const uint32_t *__restrict__ pidx, uint32_t nh, uint32_t np,
                           uint32_t *__restrict__ table)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t *hnode = table, *hpfirst = table + nh, *pnode = hpfirst + nh + 1;
    uint32_t *pfirst = pnode + np, *pn = pfirst + np;
    if (i == 0) hpfirst[nh] = np;
    if (!flag[i]) return;
    const uint32_t h = hidx[i], p0 = pidx[i], c = cnt[i];
    hnode[h] = (uint32_t)i;
    hpfirst[h] = p0;
    for (uint32_t f = 0, p = p0; f < c; f += piece, ++p) {
        pnode[p] = (uint32_t)i;
        pfirst[p] = f;
        pn[p] = c - f < piece ? c - f : piece;
    }
}

}  // namespace pdg

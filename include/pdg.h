/*
 * pdg.h -- C ABI of libpdg: the primal-dual parallel Gibbs sweep for discrete
 * pairwise MRFs with strictly positive factors (Mescheder, Nowozin, Geiger,
 * arXiv:1611.06684), built for MI355X (gfx950).
 *
 * Model.  p(x) is proportional to prod_i u_i(x_i) prod_e phi_e(x_src, x_dst),
 * x_i in {0..q_i-1}, 2 <= q_i <= q_max <= 8, every phi_e > 0 (Sec. 3, Sec. 4).
 * Each factor is decomposed into a positive mixture with one binary dual per
 * odds-ratio entry (Sec. 4.1 Lemmas, Remark and Theorem; Sec. 4.2 one-hot
 * encoding); a sweep then samples every dual given x and every node given the
 * duals (Sec. 4 Corollary, Sec. 5.1), each phase fully parallel.
 *
 * Conventions for every function:
 *   - Arguments named d_* are DEVICE pointers owned by the caller (e.g. the
 *     data_ptr() of a torch tensor on the context's device); h_* are host
 *     pointers.  The library never keeps a caller pointer after returning.
 *   - All device work is enqueued on the stream given to pdg_create, in call
 *     order.  Caller inputs must stay valid until that work completes (a
 *     stream synchronisation, or the caller's own stream ordering).
 *   - Functions return PDG_OK (0) or a negative pdg_status; no C++ exception
 *     crosses the ABI.  pdg_last_error(ctx) gives a message for the last
 *     failure on ctx.  Kernel faults are reported by the next pdg_sync.
 *   - Layouts: x is uint8 [n][C] (chain fastest); log tables are
 *     [m][q_max][q_max] row-major with row = src state; log unaries are
 *     [n][q_max]; entries beyond a node's q are ignored.  Floating inputs are
 *     float32 or float64 as chosen by pdg_config.precision.
 *   - Random numbers: Philox4x32-10 keyed by the seed, counter
 *     (id, phase, chain, call, sweep); edge draws key on the edge uid, so a
 *     trajectory does not depend on storage or edit order.
 *   - One context must not be used from two host threads at once.
 */
#ifndef PDG_H
#define PDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pdg_status;
enum {
    PDG_OK = 0,
    PDG_EINVAL = -1,     /* bad argument (null pointer, size, q, endpoint, self-loop) */
    PDG_ENOMEM = -2,     /* device or host allocation failed */
    PDG_EHIP = -3,       /* a HIP runtime call failed */
    PDG_ENOTFOUND = -4,  /* uid is not a live edge */
    PDG_ECAPACITY = -5,  /* node / edge capacity, uid space or counter range exhausted */
    PDG_ENONPOS = -6,    /* a log-factor or log-unary entry is not finite (factor not strictly positive) */
    PDG_ESTATE = -7      /* call not allowed in the current state (e.g. edit between the two phases) */
};

enum { PDG_PRECISION_F32 = 0, PDG_PRECISION_F64 = 1 };

typedef struct pdg_ctx pdg_ctx;

typedef struct {
    uint64_t seed;            /* generator key */
    int32_t n_chains;         /* C >= 1 independent chains */
    int32_t q_max;            /* 2..8, largest number of states of a node */
    int64_t node_capacity;    /* largest n accepted by pdg_set_nodes */
    int64_t edge_capacity;    /* largest number of live edges */
    int32_t precision;        /* PDG_PRECISION_F32: float32 tables and unaries, FP32 exp in
                                 the node draw; PDG_PRECISION_F64: float64 inputs and FP64
                                 exp.  Decomposition and field sums are FP64 in both. */
    int32_t reserved;         /* must be 0 */
    int64_t burn_in;          /* sweeps t <= burn_in are not counted in the marginals */
} pdg_config;

/* Create a context on HIP device `device`; all work goes to `stream`
 * (a hipStream_t; NULL = the legacy default stream). */
pdg_status pdg_create(const pdg_config *cfg, int32_t device, void *stream, pdg_ctx **out);
pdg_status pdg_destroy(pdg_ctx *ctx);

/* Nodes (once per context).  d_q: int32 [n] with 2 <= q_i <= q_max;
 * d_log_unary: [n][q_max] log u_i(a) in the configured precision. */
pdg_status pdg_set_nodes(pdg_ctx *ctx, int64_t n, const int32_t *d_q, const void *d_log_unary);

/* Insert m edges between sweeps (Sec. 4.2 decomposition runs on the new
 * edges).  d_src, d_dst: int32 [m] (src != dst, both < n); d_log_phi:
 * [m][q_max][q_max] log phi_e(a, b), row a = state of src.  d_uid_out:
 * uint64 [m] receives the library-issued uids (never reused).  O(m) work on
 * the device: no colouring, no rebuild of the incidence lists; the new entries
 * of a node follow its old ones in batch order.  Nothing changes when an
 * endpoint is out of range or equal to the other (PDG_EINVAL), a table entry
 * is not finite (PDG_ENONPOS) or capacity is short (PDG_ECAPACITY).  The call
 * synchronizes the stream (it reads back a few counters to size launches). */
pdg_status pdg_insert_edges(pdg_ctx *ctx, int64_t m, const int32_t *d_src, const int32_t *d_dst,
                            const void *d_log_phi, uint64_t *d_uid_out);

/* Remove m live edges by uid between sweeps (O(m) work on the device; the
 * freed slots are reused by later inserts under new uids).  Nothing is removed
 * if any uid is unknown or repeated (PDG_ENOTFOUND).  Synchronizes the stream.
 *
 * Failures of an edit after its checks have passed (a HIP error, or no memory
 * for a re-layout of the incidence pool, in pdg_insert_edges or
 * pdg_remove_edges) leave the edge store partly changed: the context then
 * returns PDG_ESTATE from every later call that uses the device and must be
 * destroyed.  Failures reported by the checks change nothing. */
pdg_status pdg_remove_edges(pdg_ctx *ctx, int64_t m, const uint64_t *d_uid);

/* Number of live edges, and their uids in slot order (d_uid_out: uint64 [live]). */
pdg_status pdg_num_edges(pdg_ctx *ctx, int64_t *h_live);
pdg_status pdg_live_uids(pdg_ctx *ctx, uint64_t *d_uid_out);

/* Stand-alone decomposition (Sec. 4.1, 4.2), the same kernel the insert path
 * runs.  For each of m tables (d_qs/d_qd: int32 [m] states of src/dst) writes
 * the per-edge parameter block (layout in pdg_params_layout) to d_params_out.
 * Non-finite table entries give PDG_ENONPOS.  Enqueued on `stream`, then
 * synchronized. */
pdg_status pdg_decompose(int64_t m, int32_t q_max, const int32_t *d_qs, const int32_t *d_qd,
                         const void *d_log_phi, int32_t precision, void *d_params_out,
                         void *stream);
/* Bytes per edge of the parameter block and the byte offsets of its parts,
 * for q_max (D = (q_max-1)^2, entry d = (a-1)(q_dst-1) + (b-1)):
 *   sign  uint64: bit d set when entry d's log odds ratio is negative (the
 *         row swap of the negative-determinant case, Sec. 4.1).
 *   thr   uint32 [D][2]: T+ * 256 - 1 and T- * 256, where T(k) =
 *         ceil(p(theta = 0) 2^24 - 1/2) for the dual logit t k, k in {+2, -2}
 *         (k = 0 gives T = 2^23).  The draw with 24-bit integer U is theta = 1
 *         iff U >= T(k), k = sigma (1 - 2[x_src = a]) + (1 - 2[x_dst = b]).
 *   h     double [D]: half the field increment of src state a when
 *         theta_ab = 1 (2h is the Theorem's beta1); dst state b gets 2|h| (beta2).
 *   c0    double [2][q_max-1]: field of each state >= 1 when every dual of the
 *         edge is 0 (the Theorem's alpha terms plus the table's first row /
 *         column), src side then dst side. */
pdg_status pdg_params_layout(int32_t q_max, int64_t *h_bytes_per_edge, int64_t *h_off_sign,
                             int64_t *h_off_thr, int64_t *h_off_h, int64_t *h_off_c0);

/* x(0) = floor(u q_i) for every node and chain (generator phase INIT);
 * resets the sweep counter to 0. */
pdg_status pdg_init_chains(pdg_ctx *ctx);
/* Copy a state in / out (uint8 [n][C]); pdg_set_state keeps the sweep counter.
 * pdg_set_state checks every x_i < q_i first (PDG_EINVAL and no change
 * otherwise) and synchronizes the stream. */
pdg_status pdg_set_state(pdg_ctx *ctx, const uint8_t *d_x);
pdg_status pdg_get_state(pdg_ctx *ctx, uint8_t *d_x_out);
/* Sweep counter: the last completed sweep t (0 after init).  pdg_set_sweep
 * resumes a chain at a saved counter (with pdg_set_state). */
pdg_status pdg_get_sweep(pdg_ctx *ctx, int64_t *h_t);
pdg_status pdg_set_sweep(pdg_ctx *ctx, int64_t t);

/* n_sweeps full sweeps: for t = t+1 ...: dual phase on x(t-1), then primal
 * phase, with marginal counting when t > burn_in (Sec. 5.1). */
pdg_status pdg_sweep(pdg_ctx *ctx, int64_t n_sweeps);
/* The two phases of one sweep, for teacher-forced checks and per-kernel timing:
 * pdg_dual_phase advances t and samples every dual; pdg_primal_phase samples
 * every node from those duals.  They must alternate. */
pdg_status pdg_dual_phase(pdg_ctx *ctx);
pdg_status pdg_primal_phase(pdg_ctx *ctx);

/* Duals of the last dual phase for m live uids: uint64 [m][C], bit d =
 * theta of entry d = (a-1)(q_dst-1) + (b-1). */
pdg_status pdg_get_duals(pdg_ctx *ctx, int64_t m, const uint64_t *d_uid, uint64_t *d_theta_out);

/* Log of the partition-function estimator of Sec. 5.2, one value per chain,
 * into d_out: double [C].  Called between pdg_dual_phase and pdg_primal_phase
 * (else PDG_ESTATE): x is the state the duals were drawn from and theta those
 * duals, a draw of the joint once the chain has mixed.  V(x, theta) =
 * p~(x) p~(theta) / p~(x, theta) has mean Z, and log V has mean log Z minus
 * the mutual information of x and theta, so its average over sweeps and chains
 * is a lower bound of log Z.  With the Lemma of Sec. 3, log V = log p~(x) -
 * sum_i log p(x_i | theta), p~(x) = prod_i u_i(x_i) prod_e phi_e(x_src, x_dst)
 * from the tables given at insert (kept by the library).  FP64 throughout; the
 * per-chain sums are added in a fixed order (reproducible).  Enqueued on the
 * context's stream; d_out is written when that work completes. */
pdg_status pdg_log_v(pdg_ctx *ctx, double *d_out);

/* pdg_log_v for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and result, bit for bit, with the partial sums in a static
 * workspace of 64 MiB that the library holds on every device it runs on (for
 * the process's lifetime) instead of the context's growable scratch.  Calls no
 * hipMalloc, hipFree or allocating library routine.  Needs (ceil(n/16) +
 * ceil(edge slots/64) + min(that, 1024) + 1) * 64 * ceil(C/64) * 8 bytes
 * (ceil(C/64) read as 1 for C <= 32); larger graphs get PDG_ECAPACITY and
 * nothing is launched.  Every context on a device shares that device's
 * workspace: calls on one device that overlap in time (other streams, other
 * host threads) race and must be ordered by the caller. */
pdg_status pdg_log_v_noalloc(pdg_ctx *ctx, double *d_out);

/* Marginal estimates p(x_i = a) = count / samples into d_out: double
 * [n][q_max], one correctly rounded FP64 division per entry (0 before any
 * counted sweep; entries a >= q_i are 0); *h_samples (optional) = C x counted
 * sweeps.  Synchronizes. */
pdg_status pdg_get_marginals(pdg_ctx *ctx, double *d_out, int64_t *h_samples);
/* Raw counters uint32 [n][q_max]. */
pdg_status pdg_get_counts(pdg_ctx *ctx, uint32_t *d_out, int64_t *h_samples);
pdg_status pdg_reset_marginals(pdg_ctx *ctx);

/* Replayed sweeps (HIP graphs).  pdg_graph_create captures n_sweeps full
 * sweeps (1..4096) of each of n_ctx contexts (same device and stream; for
 * example one context per state count of a batch of graphs) into one graph:
 * per sweep and context a one-thread kernel advancing that context's sweep
 * counter in device memory, then its dual and primal phase kernels, which read
 * the counter (and whether the sweep is counted) from there.  The graph holds
 * no memset or copy.  pdg_graph_launch sets each counter to the context's t
 * and replays the graph on the contexts' stream: the same draws as n_sweeps
 * pdg_sweep calls of each context, in phase launches (never the one-launch
 * form of small graphs).  A graph whose contexts have been edited since the
 * capture is refused (PDG_ESTATE); capture again.  The graph keeps the
 * contexts' buffer addresses: destroy it before the contexts. */
typedef struct pdg_graph pdg_graph;
pdg_status pdg_graph_create(pdg_ctx *const *ctxs, int32_t n_ctx, int32_t n_sweeps, pdg_graph **out);
pdg_status pdg_graph_launch(pdg_graph *graph);
pdg_status pdg_graph_destroy(pdg_graph *graph);

/* Launch parameters of the sweep kernels.  None of them changes a draw's
 * generator values; the dual's tiling changes no result at all, the hub split
 * changes the order in which a hub's field is summed (FP64 rounding only).
 *   dual_edges_per_wave     2, 4 or 8: edges one wave of the 33+-chain dual takes
 *   binary_groups_per_wave  2, 4 or 8: item groups per wave of the binary dual
 *                           (q_max 2, 8 or 16 chains)
 *   hub_threshold           nodes with more incidence entries are split into
 *                           pieces for the hub kernels (0: never)
 *   hub_piece               records per piece
 * pdg_tune times each dual tiling and each hub setting (thresholds 0, 128,
 * 256, 512, 1024; pieces 64, 128, 256) on the current graph with `reps`
 * launches each, keeps the fastest and reports the times in dual_ms and
 * primal_ms (per launch).  It runs dual and primal phases without counting and
 * restores x afterwards: the chain, its sweep counter and the counters are as
 * before.  It allocates a copy of x.  pdg_set_tuning applies given values
 * (PDG_EINVAL out of range); both refuse between the phases and make captured
 * graphs stale. */
typedef struct {
    int32_t dual_edges_per_wave;
    int32_t binary_groups_per_wave;
    int32_t hub_threshold;
    int32_t hub_piece;
    float dual_ms, primal_ms;  /* pdg_tune's measurements (-1 otherwise) */
} pdg_tuning;
pdg_status pdg_tune(pdg_ctx *ctx, int32_t reps, pdg_tuning *h_out);
pdg_status pdg_set_tuning(pdg_ctx *ctx, const pdg_tuning *h_in);
pdg_status pdg_get_tuning(pdg_ctx *ctx, pdg_tuning *h_out);

/* Wait for the context's stream and report any asynchronous kernel error. */
pdg_status pdg_sync(pdg_ctx *ctx);
/* Message of the last failure on ctx (valid until the next call on ctx);
 * with ctx == NULL, the last failure of pdg_create / pdg_decompose. */
const char *pdg_last_error(const pdg_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* PDG_H */

/*
 * pdg_oracle.c -- plain FP64 CPU oracle of the primal-dual Gibbs sweep for
 * discrete pairwise MRFs with strictly positive factors (Mescheder, Nowozin,
 * Geiger, "Probabilistic Duality for Parallel Gibbs Sampling without Graph
 * Coloring", arXiv:1611.06684).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no source, header,
 * table or helper with the GPU library, and the GPU library never calls it.
 *
 * What each part follows:
 *   orc_philox4x32_10   Philox4x32 with 10 rounds, from its published definition
 *                       (Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As
 *                       Easy as 1, 2, 3", SC'11, Sec. 3.2 / 4).
 *   orc_uniform         the counter layout and the 24-bit uniform mapping frozen
 *                       for this sampler (the paper leaves the RNG open).
 *   orc_factor2x2       Sec. 4.1: positive factorization P = B C^T of any strictly
 *                       positive 2x2 table, by the row-swap lemma (det P < 0),
 *                       the diagonal-scaling lemma (symmetrize), and the lemma
 *                       S = B B^T with the Remark's algebraic cos/sin of
 *                       phi = pi/4 - arccos(a)/2.
 *   orc_theorem_params  Sec. 4.1 Theorem: (alpha1, alpha2, q, beta1, beta2) from
 *                       B and C, so that P(y,y') is proportional to
 *                       sum_theta exp(alpha1 y + alpha2 y') exp(q theta)
 *                       exp(theta (beta1 y + beta2 y')).
 *   orc_decompose       Sec. 4.2: a q_i x q_j factor in 0-1 (one-hot) encoding.
 *                       The table is first rescaled by its first row and column
 *                       (unary factors), which turns row 0 and column 0 into
 *                       1-entries; 1-entries need no dual, every other entry
 *                       (a,b), a,b >= 1, gets one binary dual with the 2x2 table
 *                       [[1,1],[1,kappa_ab]].
 *   orc_dual_edge       Sec. 4 Corollary + Sec. 5.1: p(theta | x) factorizes over
 *                       the duals; each is a logistic draw.
 *   orc_node_logits,    Sec. 4 Corollary + Sec. 5.1: p(x | theta) factorizes over
 *   orc_primal_node     nodes; each node is a categorical draw by inverse CDF.
 *   orc_run             alternating blockwise Gibbs (Sec. 5.1): dual phase then
 *                       primal phase per sweep, marginal counting after burn-in.
 *   orc_log_v           Sec. 5.2: log of the estimator V(x, theta) =
 *                       p~(x) p~(theta) / p~(x, theta) of the partition function,
 *                       written with the Lemma of Sec. 3 as p~(x) / p(x | theta).
 *
 * Notation.  x_i in {0..q_i-1} node states; theta_{e,ab} in {0,1} the dual of
 * entry (a,b), a,b >= 1, of edge e; y = [x_src == a], y' = [x_dst == b] the
 * one-hot bits of the endpoints; Lam = log phi (row index = src state).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PHASE_INIT 0u
#define ORC_PHASE_DUAL 1u
#define ORC_PHASE_PRIMAL 2u
#define ORC_FLAG_BAND 1e-6

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon et al. 2011).  Round: two 32x32->64 products of the  */
/* even words with the multipliers, the high halves xored with the odd words   */
/* and the round key, words permuted; the key advances by the Weyl constants.  */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* One generator call keyed by the seed, counter (id_lo, id_hi, phase<<30|sub, sweep). */
static void orc_call(uint64_t seed, uint32_t phase, uint64_t id, uint32_t sub,
                     uint32_t sweep, uint32_t w[4])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {(uint32_t)id, (uint32_t)(id >> 32), (phase << 30) | sub, sweep};
    orc_philox4x32_10(ctr, key, w);
}

/* The five 24-bit integers one call yields: the top 24 bits of each word, and
 * a fifth assembled from the low bytes of words 0, 1, 2. */
static uint32_t orc_u24(const uint32_t w[4], int slot)
{
    if (slot < 4) return w[slot] >> 8;
    return ((w[0] & 0xFFu) << 16) | ((w[1] & 0xFFu) << 8) | (w[2] & 0xFFu);
}

static double orc_u24_to_unit(uint32_t u)
{
    return ((double)u + 0.5) * 0x1p-24;
}

/* Uniform in (0,1) for (phase, id, sub, sweep, slot). */
double orc_uniform(uint64_t seed, uint32_t phase, uint64_t id, uint32_t sub,
                   uint32_t sweep, int slot)
{
    uint32_t w[4];
    orc_call(seed, phase, id, sub, sweep, w);
    return orc_u24_to_unit(orc_u24(w, slot));
}

/* Many uniforms of one phase and sweep: out[k] = orc_uniform(seed, phase,
 * ids[k], subs[k], sweep, slots[k]). */
void orc_uniform_batch(uint64_t seed, uint32_t phase, uint32_t sweep, int64_t n,
                       const uint64_t *ids, const uint32_t *subs, const int32_t *slots,
                       double *out)
{
    for (int64_t k = 0; k < n; ++k)
        out[k] = orc_uniform(seed, phase, ids[k], subs[k], sweep, slots[k]);
}

/* ------------------------------------------------------------------------- */
/* Sec. 4.1: factorization of a strictly positive 2x2 table.                  */
/* P, B, C row-major: P[0]=p11, P[1]=p12, P[2]=p21, P[3]=p22.                 */
/* ------------------------------------------------------------------------- */
void orc_factor2x2(const double P[4], double B[4], double C[4])
{
    double p11 = P[0], p12 = P[1], p21 = P[2], p22 = P[3];
    int swapped = 0;
    /* Row-swap lemma: a table with negative determinant gets its rows swapped. */
    if (p11 * p22 - p12 * p21 < 0.0) {
        double t11 = p21, t12 = p22, t21 = p11, t22 = p12;
        p11 = t11; p12 = t12; p21 = t21; p22 = t22;
        swapped = 1;
    }
    /* Diagonal-scaling lemma: S = diag(1/p12, 1/p21) P is symmetric (unit off-diagonal). */
    double s11 = p11 / p12;
    double s12 = 1.0;
    double s22 = p22 / p21;
    /* Lemma S = Bt Bt^T with Bt = [[sqrt(s11) cos, sqrt(s11) sin], [sqrt(s22) sin, sqrt(s22) cos]],
     * phi = pi/4 - arccos(a)/2, a = s12 / sqrt(s11 s22); cos and sin from the Remark. */
    double a = s12 / sqrt(s11 * s22);
    if (a > 1.0) a = 1.0;
    double cphi = 0.5 * (sqrt(1.0 + a) + sqrt(1.0 - a));
    /* the Remark's sin = (sqrt(1+a) - sqrt(1-a)) / 2, multiplied through by the
     * conjugate so that it does not cancel when a is small (strong coupling) */
    double sphi = a / (sqrt(1.0 + a) + sqrt(1.0 - a));
    double r1 = sqrt(s11), r2 = sqrt(s22);
    double bt11 = r1 * cphi, bt12 = r1 * sphi, bt21 = r2 * sphi, bt22 = r2 * cphi;
    /* Undo the scaling: P = diag(p12, p21) S  =>  B = diag(p12, p21) Bt, C = Bt. */
    double b11 = p12 * bt11, b12 = p12 * bt12, b21 = p21 * bt21, b22 = p21 * bt22;
    /* Undo the swap on the rows of B. */
    if (swapped) {
        double u11 = b21, u12 = b22, u21 = b11, u22 = b12;
        b11 = u11; b12 = u12; b21 = u21; b22 = u22;
    }
    B[0] = b11; B[1] = b12; B[2] = b21; B[3] = b22;
    C[0] = bt11; C[1] = bt12; C[2] = bt21; C[3] = bt22;
}

/* Sec. 4.1 Theorem.  par = {alpha1, alpha2, q, beta1, beta2}. */
void orc_theorem_params(const double B[4], const double C[4], double par[5])
{
    double B11 = B[0], B12 = B[1], B21 = B[2], B22 = B[3];
    double C11 = C[0], C12 = C[1], C21 = C[2], C22 = C[3];
    par[0] = log(B21 / B11);
    par[1] = log(C21 / C11);
    par[2] = log((B12 * C12) / (B11 * C11));
    par[3] = log((B22 * B11) / (B12 * B21));
    par[4] = log((C22 * C11) / (C12 * C21));
}

/* ------------------------------------------------------------------------- */
/* Sec. 4.2: decomposition of every edge.                                     */
/* Lam   : [m][q_max][q_max] log-factor, row = src state, col = dst state.    */
/* par   : [m][(q_max-1)^2][5], entry d = (a-1)(q_dst-1) + (b-1).             */
/* rrow  : [m][q_max] unary part carried by the src node, rrow[a] =           */
/*         Lam(a,0) - Lam(0,0);  rcol : [m][q_max], rcol[b] = Lam(0,b)-Lam(0,0)*/
/* Returns 0, or -1 if a table entry is not finite (factor not positive).     */
/* ------------------------------------------------------------------------- */
int orc_decompose(int64_t m, int32_t q_max, const int32_t *qs, const int32_t *qd,
                  const double *Lam, double *par, double *rrow, double *rcol)
{
    const int64_t D = (int64_t)(q_max - 1) * (q_max - 1);
    for (int64_t e = 0; e < m; ++e) {
        const double *L = Lam + e * q_max * q_max;
        const int qi = qs[e], qj = qd[e];
        for (int a = 0; a < qi; ++a)
            for (int b = 0; b < qj; ++b)
                if (!isfinite(L[a * q_max + b])) return -1;
        double *pe = par + e * D * 5;
        memset(pe, 0, sizeof(double) * D * 5);
        double *rr = rrow + e * q_max, *rc = rcol + e * q_max;
        for (int a = 0; a < q_max; ++a) rr[a] = 0.0;
        for (int b = 0; b < q_max; ++b) rc[b] = 0.0;
        for (int a = 1; a < qi; ++a) rr[a] = L[a * q_max + 0] - L[0];
        for (int b = 1; b < qj; ++b) rc[b] = L[0 * q_max + b] - L[0];
        for (int a = 1; a < qi; ++a) {
            for (int b = 1; b < qj; ++b) {
                /* entry of the rescaled table phi(a,b) phi(0,0) / (phi(a,0) phi(0,b)) */
                double kappa = exp(L[a * q_max + b] + L[0] - L[a * q_max + 0] - L[b]);
                double P[4] = {1.0, 1.0, 1.0, kappa};
                double B[4], C[4];
                orc_factor2x2(P, B, C);
                orc_theorem_params(B, C, pe + ((int64_t)(a - 1) * (qj - 1) + (b - 1)) * 5);
            }
        }
    }
    return 0;
}

/* p(theta = 1 | y, y') for one dual: logistic of q + beta1 y + beta2 y'. */
double orc_dual_p1(const double par[5], int y, int yp)
{
    double logit = par[2] + par[3] * y + par[4] * yp;
    return 1.0 / (1.0 + exp(-logit));
}

/* ------------------------------------------------------------------------- */
/* Init: x_i = floor(u q_i) with u from phase INIT, sub = floor(c/4), slot c%4 */
/* ------------------------------------------------------------------------- */
void orc_init(int64_t n, int32_t C, const int32_t *q, uint64_t seed, uint8_t *x)
{
    for (int64_t i = 0; i < n; ++i)
        for (int32_t c = 0; c < C; ++c) {
            double u = orc_uniform(seed, ORC_PHASE_INIT, (uint64_t)i, (uint32_t)(c / 4), 0u, c % 4);
            x[i * C + c] = (uint8_t)floor(u * q[i]);
        }
}

/* ------------------------------------------------------------------------- */
/* Dual phase for one edge and one chain.  Draw d of chain c uses call        */
/* sub = 16 c + floor(d/5), slot d % 5.  theta bit d = 1 iff u >= p(theta=0). */
/* flag bit d set iff |u - p(theta=0)| < 1e-6.                                */
/* ------------------------------------------------------------------------- */
/* One dual given its uniform: p(theta = 0 | y, y') = 1 / (1 + exp(q + beta1 y +
 * beta2 y')) from the Theorem's parameters p = (alpha1, alpha2, q, beta1, beta2);
 * theta = 0 iff u < p(theta = 0).  *flag = [|u - p(theta = 0)| < 1e-6]. */
int orc_dual_decide(const double *p, int32_t y, int32_t yp, double u, int32_t *flag)
{
    double p0 = 1.0 / (1.0 + exp(p[2] + p[3] * y + p[4] * yp));
    *flag = fabs(u - p0) < ORC_FLAG_BAND;
    return !(u < p0);
}

void orc_dual_edge(int32_t qi, int32_t qj, int32_t q_max, const double *par_e,
                   int32_t x_src, int32_t x_dst, uint64_t uid, int32_t c,
                   uint32_t t, uint64_t seed, uint64_t *theta_out, uint64_t *flag_out)
{
    (void)q_max;
    uint64_t th = 0, fl = 0;
    uint32_t w[4] = {0, 0, 0, 0};
    for (int a = 1; a < qi; ++a) {
        for (int b = 1; b < qj; ++b) {
            int d = (a - 1) * (qj - 1) + (b - 1);
            if (d % 5 == 0)
                orc_call(seed, ORC_PHASE_DUAL, uid, (uint32_t)(16 * c + d / 5), t, w);
            double u = orc_u24_to_unit(orc_u24(w, d % 5));
            int y = (x_src == a), yp = (x_dst == b);
            int f = 0;
            if (orc_dual_decide(par_e + (int64_t)d * 5, y, yp, u, &f)) th |= (1ull << d);
            if (f) fl |= (1ull << d);
        }
    }
    *theta_out = th;
    *flag_out = fl;
}

/* ------------------------------------------------------------------------- */
/* Primal conditional of one node given the duals of its incident edges.      */
/* L(a) = lam(a) + sum over incident edges of the h- and r-terms of the bit    */
/* y_a (Theorem, Sec. 4.1) plus the rescaling unary of that edge.              */
/*   side 0 (node is src):  a>=1: rrow(a) + sum_b [alpha1 + theta_ab beta1]    */
/*   side 1 (node is dst):  b>=1: rcol(b) + sum_a [alpha2 + theta_ab beta2]    */
/* par[k] -> (q_max-1)^2 x 5 parameters of incident edge k, r[k] -> q_max.    */
/* ------------------------------------------------------------------------- */
static void orc_node_logits_p(int32_t qn, const double *lam, int64_t n_inc,
                              const int32_t *inc_side, const int32_t *inc_qother,
                              const double *const *par, const double *const *r,
                              const uint64_t *inc_theta, double *L)
{
    for (int a = 0; a < qn; ++a) L[a] = lam[a];
    for (int64_t k = 0; k < n_inc; ++k) {
        const double *pe = par[k];
        const double *rk = r[k];
        const uint64_t th = inc_theta[k];
        const int qo = inc_qother[k];
        if (inc_side[k] == 0) {
            for (int a = 1; a < qn; ++a) {
                double s = rk[a];
                for (int b = 1; b < qo; ++b) {
                    int d = (a - 1) * (qo - 1) + (b - 1);
                    int thd = (int)((th >> d) & 1u);
                    s += pe[d * 5 + 0] + thd * pe[d * 5 + 3];
                }
                L[a] += s;
            }
        } else {
            for (int b = 1; b < qn; ++b) {
                double s = rk[b];
                for (int a = 1; a < qo; ++a) {
                    int d = (a - 1) * (qn - 1) + (b - 1);
                    int thd = (int)((th >> d) & 1u);
                    s += pe[d * 5 + 1] + thd * pe[d * 5 + 4];
                }
                L[b] += s;
            }
        }
    }
}

/* Flat-array form: inc_par n_inc x (q_max-1)^2 x 5, inc_r n_inc x q_max. */
void orc_node_logits(int32_t qn, int32_t q_max, const double *lam, int64_t n_inc,
                     const int32_t *inc_side, const int32_t *inc_qother,
                     const double *inc_par, const double *inc_r,
                     const uint64_t *inc_theta, double *L)
{
    const int64_t D = (int64_t)(q_max - 1) * (q_max - 1);
    const double **pp = (const double **)malloc(sizeof(double *) * (size_t)(n_inc + 1));
    const double **rr = (const double **)malloc(sizeof(double *) * (size_t)(n_inc + 1));
    for (int64_t k = 0; k < n_inc; ++k) {
        pp[k] = inc_par + k * D * 5;
        rr[k] = inc_r + k * q_max;
    }
    orc_node_logits_p(qn, lam, n_inc, inc_side, inc_qother, pp, rr, inc_theta, L);
    free(pp);
    free(rr);
}

/* Categorical draw by inverse CDF: m = max L, w_a = exp(L(a) - m),
 * F_a = w_0 + ... + w_a, x = min{a : u F_{q-1} < F_a}.  The flag is set when u
 * lies within 1e-6 of an interior boundary F_k / F_{q-1}, k = 0..q-2. */
static int orc_categorical(int32_t qn, const double *L, double u, int *flag)
{
    double mx = L[0];
    for (int a = 1; a < qn; ++a) if (L[a] > mx) mx = L[a];
    double F[64];
    double acc = 0.0;
    for (int a = 0; a < qn; ++a) {
        acc += exp(L[a] - mx);
        F[a] = acc;
    }
    int x = qn - 1;
    for (int a = 0; a < qn; ++a)
        if (u * F[qn - 1] < F[a]) { x = a; break; }
    int f = 0;
    for (int k = 0; k + 1 < qn; ++k)
        if (fabs(u - F[k] / F[qn - 1]) < ORC_FLAG_BAND) f = 1;
    *flag = f;
    return x;
}

/* orc_categorical with its uniform given (flag bands pinned by the tests). */
int32_t orc_categorical_draw(int32_t qn, const double *L, double u, int32_t *flag_out)
{
    int f = 0;
    int x = orc_categorical(qn, L, u, &f);
    *flag_out = f;
    return x;
}

/* The node draw's uniform: call (node quad = node / 4, sub = chain c, sweep t),
 * word node mod 4. */
static int orc_primal_draw(int32_t qn, const double *L, int64_t node, int32_t c, uint32_t t,
                           uint64_t seed, int *flag)
{
    double u = orc_uniform(seed, ORC_PHASE_PRIMAL, (uint64_t)(node / 4), (uint32_t)c, t,
                           (int)(node % 4));
    return orc_categorical(qn, L, u, flag);
}

/* Flat-array form of one node's draw (for sampled checks at full size). */
void orc_primal_node(int32_t qn, int32_t q_max, const double *lam, int64_t n_inc,
                     const int32_t *inc_side, const int32_t *inc_qother,
                     const double *inc_par, const double *inc_r,
                     const uint64_t *inc_theta, int64_t node, int32_t c, uint32_t t,
                     uint64_t seed, int32_t *x_out, int32_t *flag_out)
{
    double L[64];
    orc_node_logits(qn, q_max, lam, n_inc, inc_side, inc_qother, inc_par, inc_r,
                    inc_theta, L);
    int f = 0;
    *x_out = orc_primal_draw(qn, L, node, c, t, seed, &f);
    *flag_out = f;
}

/* ------------------------------------------------------------------------- */
/* Whole-graph phases.  Layouts: x [n][C] u8; theta, dflag [m][C] u64 (bit d);*/
/* pflag [n][C] u8; counts [n][q_max] u64.                                    */
/* ------------------------------------------------------------------------- */
typedef struct {
    int64_t n, m;
    int32_t C, q_max;
    const int32_t *q;
    const double *lam;
    const int32_t *src, *dst;
    const uint64_t *uid;
    const double *par, *rrow, *rcol;
    uint64_t seed;
    /* incidence (built here): node -> list of (edge, side) */
    int64_t *off;
    int64_t *inc_e;
    int32_t *inc_s;
} orc_graph;

static int orc_graph_build(orc_graph *g)
{
    g->off = (int64_t *)calloc((size_t)g->n + 1, sizeof(int64_t));
    g->inc_e = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * g->m + 1));
    g->inc_s = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * g->m + 1));
    if (!g->off || !g->inc_e || !g->inc_s) return -1;
    for (int64_t e = 0; e < g->m; ++e) {
        g->off[g->src[e] + 1]++;
        g->off[g->dst[e] + 1]++;
    }
    for (int64_t i = 0; i < g->n; ++i) g->off[i + 1] += g->off[i];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(g->n + 1));
    if (!fill) return -1;
    memcpy(fill, g->off, sizeof(int64_t) * (size_t)g->n);
    for (int64_t e = 0; e < g->m; ++e) {
        int64_t k = fill[g->src[e]]++;
        g->inc_e[k] = e; g->inc_s[k] = 0;
        k = fill[g->dst[e]]++;
        g->inc_e[k] = e; g->inc_s[k] = 1;
    }
    free(fill);
    return 0;
}

static void orc_graph_free(orc_graph *g)
{
    free(g->off); free(g->inc_e); free(g->inc_s);
}

static void orc_dual_chain(const orc_graph *g, const uint8_t *x, int32_t c, uint32_t t,
                           uint64_t *theta, uint64_t *dflag)
{
    const int64_t D = (int64_t)(g->q_max - 1) * (g->q_max - 1);
    for (int64_t e = 0; e < g->m; ++e) {
        int32_t s = g->src[e], d = g->dst[e];
        uint64_t th, fl;
        orc_dual_edge(g->q[s], g->q[d], g->q_max, g->par + e * D * 5,
                      x[(int64_t)s * g->C + c], x[(int64_t)d * g->C + c], g->uid[e], c, t,
                      g->seed, &th, &fl);
        theta[e * g->C + c] = th;
        if (dflag) dflag[e * g->C + c] = fl;
    }
}

/* Per-node gather of the incident edges, then the node draw. */
typedef struct {
    int64_t cap;
    int32_t *sd, *qo;
    const double **pp, **rr;
    uint64_t *tt;
} orc_scratch;

static int orc_scratch_fit(orc_scratch *w, int64_t deg)
{
    if (deg <= w->cap) return 0;
    w->cap = deg;
    w->sd = (int32_t *)realloc(w->sd, sizeof(int32_t) * (size_t)deg);
    w->qo = (int32_t *)realloc(w->qo, sizeof(int32_t) * (size_t)deg);
    w->pp = (const double **)realloc((void *)w->pp, sizeof(double *) * (size_t)deg);
    w->rr = (const double **)realloc((void *)w->rr, sizeof(double *) * (size_t)deg);
    w->tt = (uint64_t *)realloc(w->tt, sizeof(uint64_t) * (size_t)deg);
    return (w->sd && w->qo && w->pp && w->rr && w->tt) ? 0 : -1;
}

static void orc_scratch_free(orc_scratch *w)
{
    free(w->sd); free(w->qo); free((void *)w->pp); free((void *)w->rr); free(w->tt);
}

static void orc_gather(const orc_graph *g, int64_t i, const uint64_t *theta, int32_t c,
                       int32_t C, orc_scratch *w)
{
    const int64_t D = (int64_t)(g->q_max - 1) * (g->q_max - 1);
    int64_t deg = g->off[i + 1] - g->off[i];
    for (int64_t k = 0; k < deg; ++k) {
        int64_t e = g->inc_e[g->off[i] + k];
        int32_t side = g->inc_s[g->off[i] + k];
        w->sd[k] = side;
        w->qo[k] = side == 0 ? g->q[g->dst[e]] : g->q[g->src[e]];
        w->pp[k] = g->par + e * D * 5;
        w->rr[k] = (side == 0 ? g->rrow : g->rcol) + e * g->q_max;
        w->tt[k] = theta[e * C + c];
    }
}

static int orc_primal_chain(const orc_graph *g, const uint64_t *theta, int32_t c,
                            uint32_t t, uint8_t *x_out, uint8_t *pflag, orc_scratch *w)
{
    for (int64_t i = 0; i < g->n; ++i) {
        int64_t deg = g->off[i + 1] - g->off[i];
        if (orc_scratch_fit(w, deg)) return -1;
        orc_gather(g, i, theta, c, g->C, w);
        double L[64];
        orc_node_logits_p(g->q[i], g->lam + i * g->q_max, deg, w->sd, w->qo, w->pp, w->rr,
                          w->tt, L);
        int f = 0;
        int xv = orc_primal_draw(g->q[i], L, i, c, t, g->seed, &f);
        x_out[i * g->C + c] = (uint8_t)xv;
        if (pflag) pflag[i * g->C + c] = (uint8_t)f;
    }
    return 0;
}

/*
 * One teacher-forced sweep t for every chain: theta = dual(x_in), x_out = primal(theta).
 * Any of dflag/pflag may be NULL.  Returns 0, -1 on allocation failure.
 */
int orc_sweep(int64_t n, int64_t m, int32_t C, int32_t q_max, const int32_t *q,
              const double *lam, const int32_t *src, const int32_t *dst,
              const uint64_t *uid, const double *par, const double *rrow,
              const double *rcol, uint64_t seed, uint32_t t, const uint8_t *x_in,
              uint64_t *theta, uint64_t *dflag, uint8_t *x_out, uint8_t *pflag)
{
    orc_graph g = {n, m, C, q_max, q, lam, src, dst, uid, par, rrow, rcol, seed, 0, 0, 0};
    if (orc_graph_build(&g)) { orc_graph_free(&g); return -1; }
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int32_t c = 0; c < C; ++c) {
        orc_scratch w = {0, 0, 0, 0, 0, 0};
        orc_dual_chain(&g, x_in, c, t, theta, dflag);
        err |= orc_primal_chain(&g, theta, c, t, x_out, pflag, &w) ? 1 : 0;
        orc_scratch_free(&w);
    }
    orc_graph_free(&g);
    return err ? -1 : 0;
}

/*
 * Primal phase of sweep t alone, from given duals theta [m][C] (teacher forcing
 * of the node draws).  pflag may be NULL.
 */
int orc_primal_phase(int64_t n, int64_t m, int32_t C, int32_t q_max, const int32_t *q,
                     const double *lam, const int32_t *src, const int32_t *dst,
                     const double *par, const double *rrow, const double *rcol,
                     uint64_t seed, uint32_t t, const uint64_t *theta, uint8_t *x_out,
                     uint8_t *pflag)
{
    orc_graph g = {n, m, C, q_max, q, lam, src, dst, 0, par, rrow, rcol, seed, 0, 0, 0};
    if (orc_graph_build(&g)) { orc_graph_free(&g); return -1; }
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int32_t c = 0; c < C; ++c) {
        orc_scratch w = {0, 0, 0, 0, 0, 0};
        err |= orc_primal_chain(&g, theta, c, t, x_out, pflag, &w) ? 1 : 0;
        orc_scratch_free(&w);
    }
    orc_graph_free(&g);
    return err ? -1 : 0;
}

/*
 * Free-running sweeps t0+1 .. t0+n_sweeps on x (in place).  After the primal
 * phase of sweep t, if t > burn_in, counts[i][x_i] += 1 for every chain.
 * n_flag_out (optional) receives the number of flagged draws (dual + primal),
 * n_draw_out (optional) the number of draws.  Chains run in parallel; each
 * chain's trajectory is independent of the thread count.
 */
int orc_run(int64_t n, int64_t m, int32_t C, int32_t q_max, const int32_t *q,
            const double *lam, const int32_t *src, const int32_t *dst,
            const uint64_t *uid, const double *par, const double *rrow,
            const double *rcol, uint64_t seed, uint32_t t0, int64_t n_sweeps,
            int64_t burn_in, uint8_t *x, uint64_t *counts, int64_t *n_flag_out,
            int64_t *n_draw_out)
{
    orc_graph g = {n, m, C, q_max, q, lam, src, dst, uid, par, rrow, rcol, seed, 0, 0, 0};
    if (orc_graph_build(&g)) { orc_graph_free(&g); return -1; }
    int64_t nflag = 0, ndraw = 0;
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : nflag, ndraw) reduction(| : err)
    for (int32_t c = 0; c < C; ++c) {
        uint64_t *theta = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(m * C + 1));
        uint64_t *dflag = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(m * C + 1));
        uint8_t *pflag = (uint8_t *)malloc((size_t)(n * C + 1));
        orc_scratch w = {0, 0, 0, 0, 0, 0};
        if (!theta || !dflag || !pflag) {
            err |= 1;
        } else {
            for (int64_t s = 1; s <= n_sweeps && !err; ++s) {
                uint32_t t = t0 + (uint32_t)s;
                orc_dual_chain(&g, x, c, t, theta, dflag);
                if (orc_primal_chain(&g, theta, c, t, x, pflag, &w)) { err |= 1; break; }
                for (int64_t e = 0; e < m; ++e) {
                    nflag += __builtin_popcountll(dflag[e * C + c]);
                    ndraw += (int64_t)(q[src[e]] - 1) * (q[dst[e]] - 1);
                }
                for (int64_t i = 0; i < n; ++i) {
                    nflag += pflag[i * C + c];
                    ndraw += 1;
                    if ((int64_t)t > burn_in && counts) {
#pragma omp atomic
                        counts[i * q_max + x[i * C + c]] += 1;
                    }
                }
            }
        }
        free(theta); free(dflag); free(pflag);
        orc_scratch_free(&w);
    }
    orc_graph_free(&g);
    if (n_flag_out) *n_flag_out = nflag;
    if (n_draw_out) *n_draw_out = ndraw;
    return err ? -1 : 0;
}

/* Logits of every node for one chain given that chain's duals theta [m]
 * (layout L [n][q_max]); used by the exact-transition tests. */
int orc_all_logits(int64_t n, int64_t m, int32_t q_max, const int32_t *q,
                   const double *lam, const int32_t *src, const int32_t *dst,
                   const double *par, const double *rrow, const double *rcol,
                   const uint64_t *theta, double *L)
{
    orc_graph g = {n, m, 1, q_max, q, lam, src, dst, 0, par, rrow, rcol, 0, 0, 0, 0};
    if (orc_graph_build(&g)) { orc_graph_free(&g); return -1; }
    orc_scratch w = {0, 0, 0, 0, 0, 0};
    int err = 0;
    for (int64_t i = 0; i < n && !err; ++i) {
        int64_t deg = g.off[i + 1] - g.off[i];
        if (orc_scratch_fit(&w, deg)) { err = 1; break; }
        orc_gather(&g, i, theta, 0, 1, &w);
        for (int a = 0; a < q_max; ++a) L[i * q_max + a] = 0.0;
        orc_node_logits_p(q[i], lam + i * q_max, deg, w.sd, w.qo, w.pp, w.rr, w.tt,
                          L + i * q_max);
    }
    orc_scratch_free(&w);
    orc_graph_free(&g);
    return err ? -1 : 0;
}

/* Sec. 5.2: V(x, theta) = p~(x) p~(theta) / p~(x, theta) has mean Z under
 * the joint, and log V has mean log Z - I(x; theta).  The Lemma of Sec. 3
 * gives p~(theta) / p~(x, theta) = 1 / p(x | theta), and p(x | theta)
 * factorizes over the nodes (Sec. 4 Corollary), so per chain c
 *   log V = sum_i lam_i(x_i) + sum_e Lam_e(x_src, x_dst)
 *           - sum_i [L_i(x_i) - log sum_{a < q_i} exp L_i(a)]
 * with L_i the node logits given theta (orc_node_logits_p).  Layouts: Lam
 * [m][q_max][q_max] (the log factor tables themselves), theta [m][C], x [n][C],
 * out [C]. */
int orc_log_v(int64_t n, int64_t m, int32_t C, int32_t q_max, const int32_t *q,
              const double *lam, const int32_t *src, const int32_t *dst, const double *Lam,
              const double *par, const double *rrow, const double *rcol,
              const uint64_t *theta, const uint8_t *x, double *out)
{
    orc_graph g = {n, m, C, q_max, q, lam, src, dst, 0, par, rrow, rcol, 0, 0, 0, 0};
    if (orc_graph_build(&g)) { orc_graph_free(&g); return -1; }
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int32_t c = 0; c < C; ++c) {
        orc_scratch w = {0, 0, 0, 0, 0, 0};
        double log_p = 0.0, log_cond = 0.0;
        for (int64_t i = 0; i < n; ++i)
            log_p += lam[i * q_max + x[i * C + c]];
        for (int64_t e = 0; e < m; ++e) {
            const int a = x[(int64_t)src[e] * C + c], b = x[(int64_t)dst[e] * C + c];
            log_p += Lam[(e * q_max + a) * q_max + b];
        }
        for (int64_t i = 0; i < n && !err; ++i) {
            int64_t deg = g.off[i + 1] - g.off[i];
            if (orc_scratch_fit(&w, deg)) { err = 1; break; }
            orc_gather(&g, i, theta, c, C, &w);
            double L[64];
            orc_node_logits_p(q[i], lam + i * q_max, deg, w.sd, w.qo, w.pp, w.rr, w.tt, L);
            double mx = L[0];
            for (int a = 1; a < q[i]; ++a) if (L[a] > mx) mx = L[a];
            double z = 0.0;
            for (int a = 0; a < q[i]; ++a) z += exp(L[a] - mx);
            log_cond += L[x[i * C + c]] - (mx + log(z));
        }
        out[c] = log_p - log_cond;
        orc_scratch_free(&w);
    }
    orc_graph_free(&g);
    return err ? -1 : 0;
}

/* Caps the threads of the OpenMP loops (timing on one core). */
void orc_set_threads(int32_t k)
{
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
#else
    (void)k;
#endif
}

/* Threads the OpenMP loops over chains use (1 without OpenMP). */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

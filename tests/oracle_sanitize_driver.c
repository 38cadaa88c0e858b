/*
 * Driver for the sanitizer build of the FP64 oracle (test infrastructure):
 * calls every exported oracle function on small random mixed-q models so that
 * AddressSanitizer and UndefinedBehaviorSanitizer see every code path
 * (decomposition, init, teacher-forced sweep, primal phase, free-running run
 * with counters, node logits, single dual / node draws, log V).  Compiled
 * together with oracle/pdg_oracle.c by tests/test_oracle_sanitizers.py; exits 0
 * when every call succeeds.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_uniform(uint64_t, uint32_t, uint64_t, uint32_t, uint32_t, int);
void orc_uniform_batch(uint64_t, uint32_t, uint32_t, int64_t, const uint64_t *, const uint32_t *,
                       const int32_t *, double *);
void orc_factor2x2(const double P[4], double B[4], double C[4]);
void orc_theorem_params(const double B[4], const double C[4], double par[5]);
int orc_decompose(int64_t, int32_t, const int32_t *, const int32_t *, const double *, double *,
                  double *, double *);
double orc_dual_p1(const double par[5], int, int);
void orc_init(int64_t, int32_t, const int32_t *, uint64_t, uint8_t *);
int orc_dual_decide(const double *, int32_t, int32_t, double, int32_t *);
void orc_dual_edge(int32_t, int32_t, int32_t, const double *, int32_t, int32_t, uint64_t, int32_t,
                   uint32_t, uint64_t, uint64_t *, uint64_t *);
void orc_node_logits(int32_t, int32_t, const double *, int64_t, const int32_t *, const int32_t *,
                     const double *, const double *, const uint64_t *, double *);
int32_t orc_categorical_draw(int32_t, const double *, double, int32_t *);
void orc_primal_node(int32_t, int32_t, const double *, int64_t, const int32_t *, const int32_t *,
                     const double *, const double *, const uint64_t *, int64_t, int32_t, uint32_t,
                     uint64_t, int32_t *, int32_t *);
int orc_sweep(int64_t, int64_t, int32_t, int32_t, const int32_t *, const double *, const int32_t *,
              const int32_t *, const uint64_t *, const double *, const double *, const double *,
              uint64_t, uint32_t, const uint8_t *, uint64_t *, uint64_t *, uint8_t *, uint8_t *);
int orc_primal_phase(int64_t, int64_t, int32_t, int32_t, const int32_t *, const double *,
                     const int32_t *, const int32_t *, const double *, const double *,
                     const double *, uint64_t, uint32_t, const uint64_t *, uint8_t *, uint8_t *);
int orc_run(int64_t, int64_t, int32_t, int32_t, const int32_t *, const double *, const int32_t *,
            const int32_t *, const uint64_t *, const double *, const double *, const double *,
            uint64_t, uint32_t, int64_t, int64_t, uint8_t *, uint64_t *, int64_t *, int64_t *);
int orc_all_logits(int64_t, int64_t, int32_t, const int32_t *, const double *, const int32_t *,
                   const int32_t *, const double *, const double *, const double *,
                   const uint64_t *, double *);
int orc_log_v(int64_t, int64_t, int32_t, int32_t, const int32_t *, const double *,
              const int32_t *, const int32_t *, const double *, const double *, const double *,
              const double *, const uint64_t *, const uint8_t *, double *);

static uint64_t rs = 88172645463325252ull;
static double rnd(void)  /* xorshift64, uniform in [0, 1) */
{
    rs ^= rs << 13;
    rs ^= rs >> 7;
    rs ^= rs << 17;
    return (double)(rs >> 11) * 0x1p-53;
}

static int check(int ok, const char *what)
{
    if (!ok) fprintf(stderr, "failed: %s\n", what);
    return ok ? 0 : 1;
}

static int run_model(int64_t n, int64_t m, int32_t qmax, int32_t C)
{
    int bad = 0;
    const int64_t D = (int64_t)(qmax - 1) * (qmax - 1);
    int32_t *q = malloc(sizeof(int32_t) * n), *src = malloc(sizeof(int32_t) * m),
            *dst = malloc(sizeof(int32_t) * m), *qs = malloc(sizeof(int32_t) * m),
            *qd = malloc(sizeof(int32_t) * m);
    double *lam = calloc((size_t)(n * qmax), sizeof(double));
    double *Lam = calloc((size_t)(m * qmax * qmax), sizeof(double));
    double *par = calloc((size_t)(m * D * 5 + 1), sizeof(double));
    double *rrow = calloc((size_t)(m * qmax), sizeof(double)), *rcol = calloc((size_t)(m * qmax), sizeof(double));
    uint64_t *uid = malloc(sizeof(uint64_t) * m);
    uint8_t *x = malloc((size_t)(n * C)), *x2 = malloc((size_t)(n * C)), *pf = malloc((size_t)(n * C));
    uint64_t *th = calloc((size_t)(m * C + 1), sizeof(uint64_t)), *df = calloc((size_t)(m * C + 1), sizeof(uint64_t));
    uint64_t *cnt = calloc((size_t)(n * qmax), sizeof(uint64_t));
    double *L = calloc((size_t)(n * qmax), sizeof(double)), *lv = calloc((size_t)C, sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        q[i] = 2 + (int32_t)(rnd() * (qmax - 1));
        for (int a = 0; a < q[i]; ++a) lam[i * qmax + a] = rnd() - 0.5;
    }
    for (int64_t e = 0; e < m; ++e) {
        src[e] = (int32_t)(rnd() * n);
        dst[e] = (int32_t)((src[e] + 1 + (int64_t)(rnd() * (n - 1))) % n);
        qs[e] = q[src[e]];
        qd[e] = q[dst[e]];
        uid[e] = (uint64_t)e + 1;
        for (int a = 0; a < qs[e]; ++a)
            for (int b = 0; b < qd[e]; ++b) Lam[(e * qmax + a) * qmax + b] = 2.0 * rnd() - 1.0;
    }
    bad += check(orc_decompose(m, qmax, qs, qd, Lam, par, rrow, rcol) == 0, "decompose");
    orc_init(n, C, q, 7, x);
    bad += check(orc_sweep(n, m, C, qmax, q, lam, src, dst, uid, par, rrow, rcol, 7, 3, x, th, df, x2,
                           pf) == 0, "sweep");
    bad += check(orc_primal_phase(n, m, C, qmax, q, lam, src, dst, par, rrow, rcol, 7, 3, th, x2,
                                  pf) == 0, "primal phase");
    bad += check(orc_log_v(n, m, C, qmax, q, lam, src, dst, Lam, par, rrow, rcol, th, x, lv) == 0,
                 "log V");
    for (int32_t c = 0; c < C; ++c) bad += check(isfinite(lv[c]), "log V finite");
    int64_t nf = 0, nd = 0;
    bad += check(orc_run(n, m, C, qmax, q, lam, src, dst, uid, par, rrow, rcol, 7, 0, 20, 5, x, cnt,
                         &nf, &nd) == 0, "run");
    uint64_t tot = 0;
    for (int64_t i = 0; i < n * qmax; ++i) tot += cnt[i];
    bad += check(tot == (uint64_t)(n * C * 15), "counter total");
    uint64_t *th1 = calloc((size_t)(m + 1), sizeof(uint64_t));
    for (int64_t e = 0; e < m; ++e) th1[e] = th[e * C];
    bad += check(orc_all_logits(n, m, qmax, q, lam, src, dst, par, rrow, rcol, th1, L) == 0, "logits");
    if (m > 0) {
        uint64_t t1 = 0, f1 = 0;
        orc_dual_edge(qs[0], qd[0], qmax, par, x[src[0] * C], x[dst[0] * C], uid[0], 0, 3, 7, &t1, &f1);
        int32_t fl = 0, xo = 0;
        orc_dual_decide(par, 1, 0, 0.5, &fl);
        int32_t side = 0, qo = qd[0];
        orc_primal_node(q[src[0]], qmax, lam + src[0] * qmax, 1, &side, &qo, par, rrow, th1, src[0],
                        0, 3, 7, &xo, &fl);
        bad += check(xo >= 0 && xo < q[src[0]], "primal node");
        double Lc[8] = {0.1, -0.3, 0.7, 0.0, 0.2, -1.0, 0.5, 0.9};
        bad += check(orc_categorical_draw(qmax, Lc, 0.37, &fl) < qmax, "categorical");
        double Lsum[8];
        orc_node_logits(q[src[0]], qmax, lam + src[0] * qmax, 1, &side, &qo, par, rrow, th1, Lsum);
    }
    free(th1);
    free(q); free(src); free(dst); free(qs); free(qd); free(lam); free(Lam); free(par);
    free(rrow); free(rcol); free(uid); free(x); free(x2); free(pf); free(th); free(df);
    free(cnt); free(L); free(lv);
    return bad;
}

int main(void)
{
    int bad = 0;
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    orc_philox4x32_10(ctr, key, out);
    uint64_t ids[3] = {1, 2, 3};
    uint32_t subs[3] = {0, 1, 2};
    int32_t slots[3] = {0, 3, 4};
    double u[3];
    orc_uniform_batch(9, 1, 2, 3, ids, subs, slots, u);
    for (int k = 0; k < 3; ++k) bad += check(u[k] > 0 && u[k] < 1, "uniform");
    double P[4] = {1.0, 2.0, 3.0, 0.5}, B[4], Cm[4], par[5];
    orc_factor2x2(P, B, Cm);
    orc_theorem_params(B, Cm, par);
    bad += check(orc_dual_p1(par, 1, 0) > 0, "dual p1");
    bad += run_model(40, 90, 2, 3);
    bad += run_model(60, 150, 5, 7);
    bad += run_model(50, 120, 8, 33);
    bad += run_model(30, 0, 4, 2);  /* no edges */
    if (bad) fprintf(stderr, "%d failures\n", bad);
    else printf("sanitized oracle run ok\n");
    return bad ? 1 : 0;
}

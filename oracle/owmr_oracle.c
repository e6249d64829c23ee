/*
 * CPU oracle for Picard iteration on the One Warehouse Multi-Retailer (OWMR) inventory
 * problem of the appendix "Extension: Inventory Control with Replenishment".
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code with the GPU path.
 *
 * Model (the appendix's problem formulation, integer units):
 *   state   s_t = (x_0, x_1 .. x_N): the central warehouse's and the retailers' stock;
 *   order   w_t: a demand of d_t units at retailer n_t;
 *   action  a_t = (q_t, reset_t): the retailer's replenishment order and the central
 *           warehouse's decision to order up to S;
 *   retailer policy (a function of the retailer's own stock and the order only): after
 *           the demand its stock is p = (x_n - d)^+; if p <= s_n it orders up to its level,
 *           q = min(S_n, c_n) - p, else q = 0 (so p + q <= c_n, q >= 0);
 *   central policy (s, S): reset iff x_0 - q <= s;
 *   transition: the retailer receives min(q, x_0): x_n <- p + min(q, x_0);
 *               x_0 <- S if reset, else (x_0 - q)^+.
 *
 *   orc_owmr_serial   the serial rollout (the answer), with R = the number of resets.
 *   orc_owmr_alg1     Algorithm 1 by brute force for any assignment of steps to processes:
 *                     in a pass every process replays the whole horizon from s_1, deciding
 *                     its own steps with the policy and applying the previous pass's cached
 *                     action (q, reset) at every other step.
 *   orc_owmr_runs     The same passes when every process owns whole retailers (the
 *                     appendix's allocation T_n), computed per process from two scans of
 *                     the cache: a process's retailers change only at its own steps, and
 *                     between two of its steps the central stock follows the cached
 *                     actions: after the last cached reset before a step it is S minus the
 *                     cached orders since, clamped at zero (clamped subtractions compose),
 *                     else the stock after the process's previous step minus the cached
 *                     orders since, clamped.  Checked against orc_owmr_alg1.
 *
 * Reading: a cached central action is the decision "order up to S", so a process applying
 * it sets x_0 = S (as the appendix's proof sketch does), not a fixed quantity.
 *
 * parity unpinned: none of the functions here; pins live in tests/test_oracle_owmr.py.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t N;                     /* retailers */
    int64_t T;                     /* orders */
    const int32_t *retailer;       /* [T] in [0, N) */
    const int32_t *demand;         /* [T] >= 0 */
    const int32_t *s_ret, *S_ret;  /* [N] reorder point, order-up-to level */
    const int32_t *cap;            /* [N] capacity c_n */
    const int32_t *x_init;         /* [N] retailer stock at t = 0 */
    int64_t s0, S0, x0_init;       /* central (s, S) and its stock at t = 0 */
} orc_owmr;

static int owmr_check(const orc_owmr *P)
{
    if (P->N <= 0 || P->T < 0 || P->S0 < 0 || P->x0_init < 0) return -1;
    for (int64_t t = 0; t < P->T; ++t)
        if (P->retailer[t] < 0 || P->retailer[t] >= P->N || P->demand[t] < 0) return -1;
    for (int n = 0; n < P->N; ++n)
        if (P->cap[n] < 0 || P->x_init[n] < 0 || P->x_init[n] > P->cap[n] || P->S_ret[n] < 0)
            return -1;
    return 0;
}

/* The retailer policy: order at stock x (before the demand) for demand d. */
static int64_t retailer_order(const orc_owmr *P, int n, int64_t x, int64_t d)
{
    const int64_t p = x > d ? x - d : 0;
    const int64_t level = P->S_ret[n] < P->cap[n] ? P->S_ret[n] : P->cap[n];
    return p <= P->s_ret[n] && level > p ? level - p : 0;
}

/* The transition for order t under action (q, reset). */
static void owmr_step(const orc_owmr *P, int64_t t, int64_t q, int reset, int64_t *x0, int64_t *x)
{
    const int n = P->retailer[t];
    const int64_t d = P->demand[t];
    const int64_t p = x[n] > d ? x[n] - d : 0;
    const int64_t got = q < *x0 ? q : *x0;
    x[n] = p + got;
    *x0 = reset ? P->S0 : (*x0 > q ? *x0 - q : 0);
}

/* Serial rollout.  q[T], reset[T] out; final_x0 (nullable), final_x[N] (nullable) out;
 * returns the number of resets R, or -1 on invalid input. */
int64_t orc_owmr_serial(const orc_owmr *P, int32_t *q, int32_t *reset, int64_t *final_x0,
                        int64_t *final_x)
{
    if (owmr_check(P)) return -1;
    int64_t *x = (int64_t *)malloc(sizeof(int64_t) * (size_t)P->N);
    if (!x) return -1;
    for (int n = 0; n < P->N; ++n) x[n] = P->x_init[n];
    int64_t x0 = P->x0_init, R = 0;
    for (int64_t t = 0; t < P->T; ++t) {
        const int n = P->retailer[t];
        const int64_t qq = retailer_order(P, n, x[n], P->demand[t]);
        const int rs = x0 - qq <= P->s0;
        q[t] = (int32_t)qq;
        reset[t] = rs;
        R += rs;
        owmr_step(P, t, qq, rs, &x0, x);
    }
    if (final_x0) *final_x0 = x0;
    if (final_x)
        for (int n = 0; n < P->N; ++n) final_x[n] = x[n];
    free(x);
    return R;
}

/* Shared fixed-point driver: pass k maps the cache (q, reset) of pass k-1 to the next;
 * stops when a pass changes nothing.  init (nullable: q = 0, no reset everywhere).
 * caches_q / caches_r (nullable, [max_passes][T]) record every pass.  Returns 0 when
 * converged within max_passes, 1 otherwise; *passes the passes run. */
typedef void (*owmr_pass_fn)(void *ctx, const int32_t *pq, const int32_t *pr, int32_t *nq,
                             int32_t *nr);

static int owmr_fixed_point(owmr_pass_fn pass, void *ctx, int64_t T, const int32_t *init_q,
                            const int32_t *init_r, int32_t max_passes, int32_t *out_q,
                            int32_t *out_r, int32_t *passes, int32_t *caches_q,
                            int32_t *caches_r)
{
    const size_t bytes = sizeof(int32_t) * (size_t)(T > 0 ? T : 1);
    int32_t *pq = (int32_t *)malloc(bytes), *pr = (int32_t *)malloc(bytes);
    int32_t *nq = (int32_t *)malloc(bytes), *nr = (int32_t *)malloc(bytes);
    if (!pq || !pr || !nq || !nr) { free(pq); free(pr); free(nq); free(nr); return -1; }
    for (int64_t t = 0; t < T; ++t) {
        pq[t] = init_q ? init_q[t] : 0;
        pr[t] = init_r ? init_r[t] : 0;
    }
    int rc = 1;
    int32_t k = 0;
    while (k < max_passes) {
        pass(ctx, pq, pr, nq, nr);
        ++k;
        if (caches_q) memcpy(caches_q + (int64_t)(k - 1) * T, nq, bytes);
        if (caches_r) memcpy(caches_r + (int64_t)(k - 1) * T, nr, bytes);
        int same = 1;
        for (int64_t t = 0; t < T && same; ++t) same = nq[t] == pq[t] && nr[t] == pr[t];
        int32_t *s;
        s = pq; pq = nq; nq = s;
        s = pr; pr = nr; nr = s;
        if (same) { rc = 0; break; }
    }
    if (T > 0) {
        memcpy(out_q, pq, bytes);
        memcpy(out_r, pr, bytes);
    }
    *passes = k;
    free(pq); free(pr); free(nq); free(nr);
    return rc;
}

/* ---------------------------------------------------------------- brute force */
typedef struct {
    const orc_owmr *P;
    const int64_t *worker;
    int64_t n_workers;
    int64_t *x;
} alg1_owmr_ctx;

static void owmr_alg1_pass(void *vctx, const int32_t *pq, const int32_t *pr, int32_t *nq,
                           int32_t *nr)
{
    const alg1_owmr_ctx *c = (const alg1_owmr_ctx *)vctx;
    const orc_owmr *P = c->P;
    for (int64_t m = 0; m < c->n_workers; ++m) {
        for (int n = 0; n < P->N; ++n) c->x[n] = P->x_init[n]; /* every view starts at s_1 */
        int64_t x0 = P->x0_init;
        for (int64_t t = 0; t < P->T; ++t) {
            int64_t q;
            int rs;
            if (c->worker[t] == m) {
                const int n = P->retailer[t];
                q = retailer_order(P, n, c->x[n], P->demand[t]);
                rs = x0 - q <= P->s0;
                nq[t] = (int32_t)q;
                nr[t] = rs;
            } else {
                q = pq[t];
                rs = pr[t];
            }
            owmr_step(P, t, q, rs, &x0, c->x);
        }
    }
}

int orc_owmr_alg1(const orc_owmr *P, const int64_t *worker, int64_t n_workers,
                  const int32_t *init_q, const int32_t *init_r, int32_t max_passes,
                  int32_t *out_q, int32_t *out_r, int32_t *passes, int32_t *caches_q,
                  int32_t *caches_r)
{
    if (owmr_check(P) || n_workers < 1) return -1;
    for (int64_t t = 0; t < P->T; ++t)
        if (worker[t] < 0 || worker[t] >= n_workers) return -1;
    alg1_owmr_ctx c = {P, worker, n_workers, (int64_t *)malloc(sizeof(int64_t) * (size_t)P->N)};
    if (!c.x) return -1;
    const int rc = owmr_fixed_point(owmr_alg1_pass, &c, P->T, init_q, init_r, max_passes, out_q,
                                    out_r, passes, caches_q, caches_r);
    free(c.x);
    return rc;
}

/* ---------------------------------------------------------------- per-process form */
typedef struct {
    const orc_owmr *P;
    const int64_t *group;   /* [N] process of each retailer */
    int64_t n_groups;
    int64_t *Q;             /* [T+1] prefix sums of the cached orders */
    int64_t *LR;            /* [T+1] last cached reset before t, or -1 */
    int64_t *x;             /* [N] */
    int64_t *x0v, *last;    /* [n_groups] a process's central stock after its last step */
} runs_owmr_ctx;

static void owmr_runs_pass(void *vctx, const int32_t *pq, const int32_t *pr, int32_t *nq,
                           int32_t *nr)
{
    const runs_owmr_ctx *c = (const runs_owmr_ctx *)vctx;
    const orc_owmr *P = c->P;
    c->Q[0] = 0;
    c->LR[0] = -1;
    for (int64_t t = 0; t < P->T; ++t) {
        c->Q[t + 1] = c->Q[t] + pq[t];
        c->LR[t + 1] = pr[t] ? t : c->LR[t];
    }
    for (int n = 0; n < P->N; ++n) c->x[n] = P->x_init[n];
    for (int64_t m = 0; m < c->n_groups; ++m) {
        c->x0v[m] = P->x0_init;
        c->last[m] = -1; /* no step yet: the stock at t = 0 */
    }
    /* every process's steps in time order (the processes are independent; one sweep over
       t visits each process's steps in its own order) */
    for (int64_t t = 0; t < P->T; ++t) {
        const int n = P->retailer[t];
        const int64_t m = c->group[n];
        const int64_t a = c->last[m] + 1; /* others' steps a .. t-1 since m's last step */
        int64_t x0;
        if (c->LR[t] >= a) { /* a cached reset at r in [a, t): S, then the orders after r */
            const int64_t r = c->LR[t];
            const int64_t v = P->S0 - (c->Q[t] - c->Q[r + 1]);
            x0 = v > 0 ? v : 0;
        } else {
            const int64_t v = c->x0v[m] - (c->Q[t] - c->Q[a]);
            x0 = v > 0 ? v : 0;
        }
        const int64_t q = retailer_order(P, n, c->x[n], P->demand[t]);
        const int rs = x0 - q <= P->s0;
        nq[t] = (int32_t)q;
        nr[t] = rs;
        const int64_t d = P->demand[t];
        const int64_t p = c->x[n] > d ? c->x[n] - d : 0;
        c->x[n] = p + (q < x0 ? q : x0);
        c->x0v[m] = rs ? P->S0 : (x0 > q ? x0 - q : 0);
        c->last[m] = t;
    }
}

int orc_owmr_runs(const orc_owmr *P, const int64_t *group, int64_t n_groups,
                  const int32_t *init_q, const int32_t *init_r, int32_t max_passes,
                  int32_t *out_q, int32_t *out_r, int32_t *passes, int32_t *caches_q,
                  int32_t *caches_r)
{
    if (owmr_check(P) || n_groups < 1) return -1;
    for (int n = 0; n < P->N; ++n)
        if (group[n] < 0 || group[n] >= n_groups) return -1;
    runs_owmr_ctx c = {P, group, n_groups,
                       (int64_t *)malloc(sizeof(int64_t) * (size_t)(P->T + 1)),
                       (int64_t *)malloc(sizeof(int64_t) * (size_t)(P->T + 1)),
                       (int64_t *)malloc(sizeof(int64_t) * (size_t)P->N),
                       (int64_t *)malloc(sizeof(int64_t) * (size_t)n_groups),
                       (int64_t *)malloc(sizeof(int64_t) * (size_t)n_groups)};
    int rc = -1;
    if (c.Q && c.LR && c.x && c.x0v && c.last)
        rc = owmr_fixed_point(owmr_runs_pass, &c, P->T, init_q, init_r, max_passes, out_q,
                              out_r, passes, caches_q, caches_r);
    free(c.Q); free(c.LR); free(c.x); free(c.x0v); free(c.last);
    return rc;
}

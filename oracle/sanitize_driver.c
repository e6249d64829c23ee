/*
 * Sanitizer driver for the CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY (built by tests/test_oracle_sanitize.py with gcc
 * -fsanitize=address,undefined together with picard_oracle.c, run on the host).
 *
 * Calls every exported oracle function on small random instances (both policies, one and
 * two hidden layers, capacities, warm caches, pass limits below convergence) so that
 * AddressSanitizer and UndefinedBehaviorSanitizer see every code path: out-of-bounds
 * reads or writes, leaks, signed overflow, bad shifts.  It also checks the results that
 * must agree (the brute-force Algorithm 1 against the run form and the serial rollout),
 * and exits non-zero on any disagreement or failed call.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t N, K, R;
    int64_t T;
    const int32_t *sku, *region, *qty;
    const int32_t *x0;
    const int32_t *cost;
    const float *params;
    int32_t hidden, n_hidden_layers;
    uint64_t rng_seed;
    int32_t traj;
} orc_problem;

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]);
double orc_uniform(uint64_t seed, int32_t traj, int64_t t, int32_t w);
double orc_gumbel(uint64_t seed, int32_t traj, int64_t t, int32_t w);
int64_t orc_param_count(int32_t R, int32_t H, int32_t L);
int orc_serial(const orc_problem *P, int32_t *actions, int32_t *shipped, int32_t *final_inv,
               double *z1, double *z2);
int orc_eval_at(const orc_problem *P, const int32_t *actions, int32_t *choice, double *z1,
                double *z2, int32_t *n_feasible);
int orc_eval_at_range(const orc_problem *P, const int32_t *actions, int64_t lo, int64_t hi,
                      int32_t *choice, double *z1, double *z2, int32_t *n_feasible);
int orc_reinforce_range(const orc_problem *P, const int32_t *actions, const double *adv,
                        int64_t lo, int64_t hi, double *logp, double *grad, double *objective);
int orc_policy_at(const orc_problem *P, int64_t n, const int64_t *ts, const int32_t *x_rows,
                  int32_t *choice, double *z1, double *z2);
int orc_alg1(const orc_problem *P, const int64_t *worker, int64_t n_workers,
             const int32_t *init_cache, int32_t max_passes, int32_t *final_cache,
             int32_t *passes, int32_t *caches);
int orc_picard_runs(const orc_problem *P, const int64_t *worker, const int32_t *init_cache,
                    int32_t max_passes, int32_t *final_cache, int32_t *passes,
                    int64_t *changed, int32_t *caches);
int orc_reinforce(const orc_problem *P, const int32_t *actions, const double *adv,
                  double *logp, double *grad, double *objective);
int orc_mlp_scores(const orc_problem *P, int32_t r, const int32_t *x, double *s);
typedef struct {
    int32_t gnum, gden, glow;
    const int32_t *bid_inv, *bid_cap;
} orc_cap_policy;
int orc_serial_cap(const orc_problem *P, const int32_t *cap0, const orc_cap_policy *pol,
                   int32_t *actions, int32_t *final_inv, int32_t *final_cap);
int orc_alg1_cap(const orc_problem *P, const int32_t *cap0, const orc_cap_policy *pol,
                 const int64_t *worker, int64_t n_workers, const int32_t *init_cache,
                 int32_t max_passes, int32_t *final_cache, int32_t *passes, int32_t *caches);
int orc_picard_timeblocks_cap(const orc_problem *P, const int32_t *cap0,
                              const orc_cap_policy *pol, int64_t B, const int32_t *init_cache,
                              int32_t max_passes, int32_t *final_cache, int32_t *passes,
                              int64_t *changed, int32_t *caches);

static uint64_t rs = 88172645463325252ull;
static uint32_t rnd(void) /* xorshift64 */
{
    rs ^= rs << 13;
    rs ^= rs >> 7;
    rs ^= rs << 17;
    return (uint32_t)(rs >> 32);
}
static int32_t uni(int32_t lo, int32_t hi) { return lo + (int32_t)(rnd() % (uint32_t)(hi - lo + 1)); }

static int fails = 0;
#define CHECK(cond, what)                                                                    \
    do {                                                                                     \
        if (!(cond)) {                                                                       \
            fprintf(stderr, "FAIL case %d: %s\n", ci, what);                                 \
            ++fails;                                                                         \
        }                                                                                    \
    } while (0)

int main(void)
{
    const int MAXP = 64;
    for (int ci = 0; ci < 60; ++ci) {
        const int mlp = ci % 3 == 1, layers = ci % 6 == 1 ? 1 : 2, cap = ci % 3 == 2;
        const int32_t N = uni(1, 6), K = uni(1, 4), R = uni(1, 4);
        const int64_t T = uni(0, 40);
        int32_t *sku = malloc(sizeof(int32_t) * (T + 1)), *region = malloc(sizeof(int32_t) * (T + 1));
        int32_t *qty = malloc(sizeof(int32_t) * (T + 1));
        int32_t *x0 = malloc(sizeof(int32_t) * K * N), *cost = malloc(sizeof(int32_t) * N * R);
        for (int64_t t = 0; t < T; ++t) {
            sku[t] = uni(0, K - 1);
            region[t] = uni(0, R - 1);
            qty[t] = cap ? 1 : uni(1, 3);
        }
        for (int i = 0; i < K * N; ++i) x0[i] = uni(0, 4);
        for (int i = 0; i < N * R; ++i) cost[i] = uni(1, 5);
        const int64_t np = orc_param_count(R, 64, layers);
        float *params = NULL;
        if (mlp) {
            params = malloc(sizeof(float) * np);
            for (int64_t i = 0; i < np; ++i) params[i] = ((float)(rnd() % 2001) - 1000.f) / 4000.f;
        }
        orc_problem P = {N, K, R, T, sku, region, qty, x0, cost, params, 64, layers,
                         ((uint64_t)rnd() << 32) | rnd(), ci};
        int32_t *act = malloc(sizeof(int32_t) * (T + 1)), *sh = malloc(sizeof(int32_t) * (T + 1));
        int32_t *fin = malloc(sizeof(int32_t) * K * N), *ch = malloc(sizeof(int32_t) * (T + 1));
        int32_t *nf = malloc(sizeof(int32_t) * (T + 1));
        double *z1 = malloc(sizeof(double) * (T + 1)), *z2 = malloc(sizeof(double) * (T + 1));
        int64_t *worker = malloc(sizeof(int64_t) * (T + 1));
        int32_t *init = malloc(sizeof(int32_t) * (T + 1)), *fc = malloc(sizeof(int32_t) * (T + 1));
        int32_t *fc2 = malloc(sizeof(int32_t) * (T + 1));
        int32_t *caches = malloc(sizeof(int32_t) * (T + 1) * MAXP);
        int32_t *caches2 = malloc(sizeof(int32_t) * (T + 1) * MAXP);
        int64_t *changed = malloc(sizeof(int64_t) * MAXP);
        const int64_t nw = uni(1, 5);
        for (int64_t t = 0; t < T; ++t) {
            worker[t] = uni(0, (int32_t)nw - 1);
            init[t] = uni(-1, N - 1);
        }
        if (!cap) {
            CHECK(orc_serial(&P, act, sh, fin, z1, z2) == 0, "orc_serial");
            CHECK(orc_eval_at(&P, act, ch, z1, z2, nf) == 0, "orc_eval_at");
            for (int64_t t = 0; t < T; ++t) CHECK(ch[t] == act[t], "eval_at at the serial actions");
            {   /* the same over two windows, and the policy at the states of a replay */
                const int64_t mid = T / 2;
                int32_t *ch2 = malloc(sizeof(int32_t) * (T + 1));
                CHECK(orc_eval_at_range(&P, act, 0, mid, ch2, NULL, NULL, NULL) == 0 &&
                      orc_eval_at_range(&P, act, mid, T, ch2, NULL, NULL, NULL) == 0, "windows");
                for (int64_t t = 0; t < T; ++t) CHECK(ch2[t] == act[t], "windowed eval_at");
                int32_t *rows = malloc(sizeof(int32_t) * (T + 1) * N), *xr = malloc(sizeof(int32_t) * K * N);
                int64_t *ts = malloc(sizeof(int64_t) * (T + 1));
                memcpy(xr, x0, sizeof(int32_t) * K * N);
                for (int64_t t = 0; t < T; ++t) {
                    int32_t *xk = xr + (int64_t)sku[t] * N;
                    memcpy(rows + t * N, xk, sizeof(int32_t) * N);
                    ts[t] = t;
                    if (act[t] >= 0) xk[act[t]] -= xk[act[t]] < qty[t] ? xk[act[t]] : qty[t];
                }
                CHECK(orc_policy_at(&P, T, ts, rows, ch2, NULL, NULL) == 0, "orc_policy_at");
                for (int64_t t = 0; t < T; ++t) CHECK(ch2[t] == act[t], "policy at replayed states");
                free(ch2); free(rows); free(xr); free(ts);
            }
            int32_t p1 = 0, p2 = 0;
            const int32_t *ic = ci % 2 ? init : NULL;
            const int r1 = orc_alg1(&P, worker, nw, ic, MAXP, fc, &p1, caches);
            const int r2 = orc_picard_runs(&P, worker, ic, MAXP, fc2, &p2, changed, caches2);
            CHECK(r1 == 0 && r2 == 0 && p1 == p2, "alg1 and run form converge together");
            CHECK(memcmp(caches, caches2, sizeof(int32_t) * T * p1) == 0, "per-pass caches");
            CHECK(memcmp(fc, act, sizeof(int32_t) * T) == 0, "fixed point is the serial rollout");
            if (p1 > 1) { /* a pass limit below convergence */
                CHECK(orc_alg1(&P, worker, nw, ic, p1 - 1, fc, &p2, NULL) == 1, "alg1 limit");
                CHECK(orc_picard_runs(&P, worker, ic, p1 - 1, fc2, &p2, NULL, NULL) == 1, "runs limit");
            }
            if (mlp) {
                double *adv = malloc(sizeof(double) * (T + 1)), *lp = malloc(sizeof(double) * (T + 1));
                double *g = malloc(sizeof(double) * np), obj = 0.0;
                for (int64_t t = 0; t < T; ++t) adv[t] = ((double)(rnd() % 200) - 100.0) / 50.0;
                CHECK(orc_reinforce(&P, act, adv, lp, g, &obj) == 0, "orc_reinforce");
                double obj2 = 0.0;
                CHECK(orc_reinforce_range(&P, act, adv, T / 3, T, lp, g, &obj2) == 0,
                      "orc_reinforce_range");
                CHECK(isfinite(obj), "finite objective");
                double *s = malloc(sizeof(double) * N);
                CHECK(orc_mlp_scores(&P, 0, x0, s) == 0, "orc_mlp_scores");
                free(adv); free(lp); free(g); free(s);
            }
        } else {
            int32_t *cap0 = malloc(sizeof(int32_t) * N), *fcap = malloc(sizeof(int32_t) * N);
            for (int w = 0; w < N; ++w) cap0[w] = uni(0, 6);
            const int32_t gnum = ci % 2 ? uni(1, 3) : 0, gden = uni(1, 2);
            const int32_t glow = ci % 3 == 1 ? uni(1, 4) : 0;
            int32_t *bi = malloc(sizeof(int32_t) * K * N), *bc = malloc(sizeof(int32_t) * N);
            for (int64_t i = 0; i < (int64_t)K * N; ++i) bi[i] = uni(0, 4) - 2;
            for (int w = 0; w < N; ++w) bc[w] = uni(0, 3);
            const int bid = !gnum && ci % 5 == 2;
            const orc_cap_policy pol = {gnum, gden, glow, bid ? bi : NULL, bid ? bc : NULL};
            CHECK(orc_serial_cap(&P, cap0, &pol, act, fin, fcap) == 0, "orc_serial_cap");
            int32_t p1 = 0, p2 = 0;
            const int64_t B = uni(1, 7);
            for (int64_t t = 0; t < T; ++t) worker[t] = t / B;
            const int64_t nb = T > 0 ? (T + B - 1) / B : 1;
            const int32_t *ic = ci % 4 == 3 ? init : NULL;
            const int r1 = orc_alg1_cap(&P, cap0, &pol, worker, nb, ic, MAXP, fc, &p1, caches);
            const int r2 = orc_picard_timeblocks_cap(&P, cap0, &pol, B, ic, MAXP, fc2, &p2,
                                                     changed, caches2);
            CHECK(r1 == r2 && p1 == p2, "alg1_cap and the time-block replay agree");
            CHECK(memcmp(caches, caches2, sizeof(int32_t) * T * p1) == 0, "per-pass caches (cap)");
            if (r1 == 0) CHECK(memcmp(fc, act, sizeof(int32_t) * T) == 0, "cap fixed point is serial");
            free(cap0); free(fcap); free(bi); free(bc);
        }
        uint32_t c[4] = {rnd(), rnd(), rnd(), rnd()}, k[2] = {rnd(), rnd()}, o[4];
        orc_philox4x32_10(c, k, o);
        const double u = orc_uniform(P.rng_seed, ci, T, N - 1), g = orc_gumbel(P.rng_seed, ci, T, 0);
        CHECK(u > 0.0 && u < 1.0 && isfinite(g), "uniform and gumbel");
        free(sku); free(region); free(qty); free(x0); free(cost); free(params);
        free(act); free(sh); free(fin); free(ch); free(nf); free(z1); free(z2);
        free(worker); free(init); free(fc); free(fc2); free(caches); free(caches2); free(changed);
    }
    if (fails) {
        fprintf(stderr, "%d check(s) failed\n", fails);
        return 1;
    }
    printf("sanitize driver: all oracle calls clean\n");
    return 0;
}

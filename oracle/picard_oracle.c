/*
 * CPU oracle for Picard policy simulation on the fulfillment problem.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code with the GPU path.
 *
 * Everything here is written to be read against the paper, not to be fast:
 *
 *   orc_serial        the serial rollout that defines the answer (Section 2, problem
 *                     statement: a_t = pi(s_t, w_t), s_{t+1} = f(s_t, a_t, w_t)), with the
 *                     FO transition of Section 3 (no node capacity).
 *   orc_alg1          Algorithm 1 (the Picard iteration) by brute force: in a pass every
 *                     process has its own view of the whole horizon (process_view, the
 *                     same replay that gives the serial rollout), and run_passes iterates
 *                     the pass map to its fixed point.  O(P*T*N) per pass: tiny
 *                     instances only.
 *   orc_picard_runs   The same passes, computed per SKU: by inventory independence
 *                     (Assumption 1) and with no capacity, SKUs never interact.  A
 *                     process reaching one of its runs of a SKU has applied the cached
 *                     actions of the other processes' earlier orders and its own fresh
 *                     actions of its earlier runs, so it sees the initial inventory
 *                     minus both consumptions, clamped at zero (clamp: max(0,
 *                     max(0, x-a) - b) = max(0, x-a-b)).  Checked against orc_alg1.
 *   orc_eval_at       The policy evaluated at every step of a GIVEN action sequence
 *                     (the state that sequence induces), for self-consistency checks.
 *   orc_reinforce     FP64 REINFORCE surrogate sum_t A_t log pi(a_t | s_t) and its
 *                     gradient by hand-written backpropagation (Section 4.2 trains the
 *                     policy by policy gradient).
 *   orc_serial_cap, orc_alg1_cap, orc_picard_timeblocks_cap
 *                     The serial rollout and Algorithm 1 with node capacity (Section 3,
 *                     the full FO state (x_t, c_t)), greedy policy, unit demand; the
 *                     last one computes Algorithm 1's passes for the partition into
 *                     time blocks in one replay per pass.  Checked against each other
 *                     and against the no-capacity functions where they coincide.
 *   orc_philox4x32_10 Philox4x32-10 from Salmon, Moraes, Dror and Shaw, "Parallel random
 *                     numbers: as easy as 1, 2, 3" (SC'11): the counter-based generator
 *                     that supplies the learned policy's Gumbel noise (the paper lets the
 *                     disturbance w_t carry the policy's own randomness, Section 2).
 *
 * Semantics fixed by this oracle (readings of the paper, see the design notes):
 *   - a warehouse w is feasible for an order of SKU k iff x[k][w] > 0 (Section 3 action
 *     set); an order of quantity q sent to w ships min(q, x[k][w]); the rest is lost;
 *   - greedy policy: the feasible warehouse of least cost[w][region], lowest index on
 *     ties, lost sale iff none is feasible (Section 3.1 greedy policy, with inventory in
 *     place of capacity);
 *   - learned policy: z_w = mlp(cost[w][r], log1p(x[k][w]), E[r]) + Gumbel(t, traj, w),
 *     argmax over feasible w, lowest index on exact ties;
 *   - "passes" is the k at which Algorithm 1 returns (alpha^k == alpha^{k-1}).
 *
 * parity unpinned: none of the functions here; pins live in tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define LOST (-1)

typedef struct {
    int32_t N, K, R;
    int64_t T;
    const int32_t *sku, *region, *qty; /* [T], time order */
    const int32_t *x0;                 /* [K][N] */
    const int32_t *cost;               /* [N][R] */
    const float *params;               /* NULL: greedy policy; else learned policy */
    int32_t hidden, n_hidden_layers;
    uint64_t rng_seed;
    int32_t traj; /* trajectory index inside its batch (part of the Philox counter) */
} orc_problem;

/* ------------------------------------------------------------------------------------
 * Philox4x32-10 (SC'11).  Round: two 32x32->64 products of counter words 0 and 2 with
 * the round multipliers; the new counter is (hi1^c1^k0, lo1, hi0^c3^k1, lo0).  The key
 * is bumped by the Weyl constants between rounds.
 * ---------------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in (0,1): 23 random bits, centred: ((u >> 9) + 0.5) * 2^-23.  Every value is
 * exactly representable in binary32, so both precisions start from the same U. */
double orc_uniform(uint64_t seed, int32_t traj, int64_t t, int32_t w)
{
    uint32_t ctr[4] = {(uint32_t)t, (uint32_t)traj, (uint32_t)w >> 2, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    uint32_t u = out[w & 3];
    return ((double)(u >> 9) + 0.5) * (1.0 / 8388608.0);
}

double orc_gumbel(uint64_t seed, int32_t traj, int64_t t, int32_t w)
{
    return -log(-log(orc_uniform(seed, traj, t, w)));
}

/* ------------------------------------------------------------------------------------
 * The learned score in FP64.  Parameter pack (float32 on input):
 *   E[R][16] | W1[H][18] | b1[H] | (W2[H][H] | b2[H] if two hidden layers) | w3[H] | b3
 * Features f = [cost, log1p(x), E[r][0..15]]; h1 = relu(W1 f + b1);
 * h2 = relu(W2 h1 + b2); s = w3 . h_last + b3.
 * ---------------------------------------------------------------------------------- */
typedef struct {
    int H, L, R;
    double *E, *W1, *b1, *W2, *b2, *w3, b3;
    double *buf;
} mlp64;

static int64_t param_count(int R, int H, int L)
{
    int64_t n = (int64_t)R * 16 + (int64_t)H * 18 + H;
    if (L == 2) n += (int64_t)H * H + H;
    return n + H + 1;
}

int64_t orc_param_count(int32_t R, int32_t H, int32_t L) { return param_count(R, H, L); }

static int mlp_load(mlp64 *m, const orc_problem *P)
{
    m->H = P->hidden; m->L = P->n_hidden_layers; m->R = P->R;
    if (m->H <= 0 || (m->L != 1 && m->L != 2)) return -1;
    int64_t n = param_count(m->R, m->H, m->L);
    m->buf = (double *)malloc(sizeof(double) * (size_t)n);
    if (!m->buf) return -1;
    for (int64_t i = 0; i < n; ++i) m->buf[i] = (double)P->params[i];
    double *p = m->buf;
    m->E = p; p += (int64_t)m->R * 16;
    m->W1 = p; p += (int64_t)m->H * 18;
    m->b1 = p; p += m->H;
    if (m->L == 2) { m->W2 = p; p += (int64_t)m->H * m->H; m->b2 = p; p += m->H; }
    else { m->W2 = NULL; m->b2 = NULL; }
    m->w3 = p; p += m->H;
    m->b3 = *p;
    return 0;
}

static void mlp_free(mlp64 *m) { free(m->buf); m->buf = NULL; }

/* Forward for one (order, warehouse) row.  pre1/h1/pre2/h2 may be NULL when the caller
 * does not need the activations (they are used by the backward pass). */
static double mlp_forward(const mlp64 *m, double cost, double inv, int r, double *f,
                          double *pre1, double *h1, double *pre2, double *h2)
{
    const int H = m->H;
    double f_loc[18], a1[1024], z1[1024], a2[1024], z2[1024];
    if (!f) f = f_loc;
    if (!pre1) pre1 = a1;
    if (!h1) h1 = z1;
    if (!pre2) pre2 = a2;
    if (!h2) h2 = z2;
    f[0] = cost;
    f[1] = log1p(inv);
    for (int i = 0; i < 16; ++i) f[2 + i] = m->E[r * 16 + i];
    for (int j = 0; j < H; ++j) {
        double acc = m->b1[j];
        for (int i = 0; i < 18; ++i) acc += m->W1[j * 18 + i] * f[i];
        pre1[j] = acc;
        h1[j] = acc > 0.0 ? acc : 0.0;
    }
    const double *hl = h1;
    if (m->L == 2) {
        for (int j = 0; j < H; ++j) {
            double acc = m->b2[j];
            for (int i = 0; i < H; ++i) acc += m->W2[j * H + i] * h1[i];
            pre2[j] = acc;
            h2[j] = acc > 0.0 ? acc : 0.0;
        }
        hl = h2;
    }
    double s = m->b3;
    for (int j = 0; j < H; ++j) s += m->w3[j] * hl[j];
    return s;
}

/* ------------------------------------------------------------------------------------
 * The policy pi(s_t, w_t) for one order.  `x` is the inventory row of the order's SKU.
 * Returns the chosen warehouse or LOST; for the learned policy also the two largest
 * perturbed scores among feasible warehouses (z1 >= z2; -inf when absent).
 * ---------------------------------------------------------------------------------- */
static int32_t policy(const orc_problem *P, const mlp64 *m, int64_t t, const int32_t *x,
                      double *z1, double *z2)
{
    const int N = P->N, R = P->R;
    const int r = P->region[t];
    int32_t best = LOST;
    if (!P->params) {
        int32_t best_cost = 0;
        for (int w = 0; w < N; ++w) {
            if (x[w] <= 0) continue;
            int32_t c = P->cost[w * R + r];
            if (best == LOST || c < best_cost) { best = w; best_cost = c; }
        }
        return best;
    }
    double top1 = -INFINITY, top2 = -INFINITY;
    for (int w = 0; w < N; ++w) {
        if (x[w] <= 0) continue;
        double s = mlp_forward(m, (double)P->cost[w * R + r], (double)x[w], r, NULL, NULL,
                               NULL, NULL, NULL);
        double z = s + orc_gumbel(P->rng_seed, P->traj, t, w);
        if (best == LOST || z > top1) { top2 = top1; top1 = z; best = w; }
        else if (z > top2) top2 = z;
    }
    if (z1) *z1 = top1;
    if (z2) *z2 = top2;
    return best;
}

/* f(s, a, w) restricted to the order's SKU row: ship min(q, x[a]). Returns shipped. */
static int32_t transition(int32_t *x, int32_t a, int32_t q)
{
    if (a == LOST) return 0;
    int32_t sh = x[a] < q ? x[a] : q;
    x[a] -= sh;
    return sh;
}

static int check_problem(const orc_problem *P)
{
    if (P->N <= 0 || P->K <= 0 || P->R <= 0 || P->T < 0) return -1;
    for (int64_t t = 0; t < P->T; ++t) {
        if (P->sku[t] < 0 || P->sku[t] >= P->K) return -1;
        if (P->region[t] < 0 || P->region[t] >= P->R) return -1;
        if (P->qty[t] < 1) return -1;
    }
    for (int64_t i = 0; i < (int64_t)P->K * P->N; ++i)
        if (P->x0[i] < 0) return -1;
    return 0;
}

/* ------------------------------------------------------------------------------------
 * One process's view of the horizon (no capacity).  The view starts from s_1 and takes
 * the orders in time order.  An order the process owns (owner == NULL: every order) is
 * decided by the policy at the state the view has reached, and the decision goes to
 * decided[t]; any other order applies given[t], or the lost sale when given[t] is not
 * feasible at that state (the lost sale always is).  shipped/z1/z2 (nullable) receive
 * the units shipped by the view and, for the learned policy, the top two perturbed
 * scores of every decided order.  x is scratch of K*N entries.
 * ---------------------------------------------------------------------------------- */
static void process_view(const orc_problem *P, const mlp64 *m, const int64_t *owner,
                         int64_t self, const int32_t *given, int32_t *decided, int32_t *x,
                         int32_t *shipped, double *z1, double *z2)
{
    const int N = P->N;
    memcpy(x, P->x0, sizeof(int32_t) * (size_t)P->K * N); /* every view starts at s_1 */
    for (int64_t t = 0; t < P->T; ++t) {
        int32_t *xk = x + (int64_t)P->sku[t] * N;
        int32_t a;
        if (!owner || owner[t] == self) {
            double a1 = -INFINITY, a2 = -INFINITY;
            a = policy(P, m, t, xk, &a1, &a2);
            decided[t] = a;
            if (z1) z1[t] = a1;
            if (z2) z2[t] = a2;
        } else {
            a = given[t];
            if (a != LOST && (a < 0 || a >= N || xk[a] <= 0)) a = LOST;
        }
        const int32_t sh = transition(xk, a, P->qty[t]);
        if (shipped) shipped[t] = sh;
    }
}

/* ------------------------------------------------------------------------------------
 * Serial rollout (the definition of the answer): the view of a process that owns
 * every order.
 * ---------------------------------------------------------------------------------- */
int orc_serial(const orc_problem *P, int32_t *actions, int32_t *shipped, int32_t *final_inv,
               double *z1, double *z2)
{
    if (check_problem(P)) return -1;
    const int N = P->N;
    mlp64 m = {0};
    if (P->params && mlp_load(&m, P)) return -1;
    int32_t *x = (int32_t *)malloc(sizeof(int32_t) * (size_t)P->K * N);
    if (!x) { mlp_free(&m); return -1; }
    process_view(P, &m, NULL, 0, NULL, actions, x, shipped, z1, z2);
    if (final_inv) memcpy(final_inv, x, sizeof(int32_t) * (size_t)P->K * N);
    free(x);
    mlp_free(&m);
    return 0;
}

/* ------------------------------------------------------------------------------------
 * Fixed-point driver shared by the Picard oracles.  A pass maps the previous cache to
 * the next one; passes run from alpha^0 (init_cache, or the lost sale everywhere) until
 * one returns its own input (Algorithm 1's termination test) or max_passes is reached.
 * caches (nullable) receives alpha^1 .. alpha^passes, T entries each; changed
 * (nullable) the number of steps each pass changed.  Returns 0 when converged (passes =
 * the k with alpha^k == alpha^{k-1}), 1 when max_passes was reached first
 * (final_cache then holds alpha^max_passes), -1 when out of memory.
 * ---------------------------------------------------------------------------------- */
typedef void (*pass_fn)(void *ctx, const int32_t *prev, int32_t *next);

static int run_passes(pass_fn pass, void *ctx, int64_t T, const int32_t *init_cache,
                      int32_t max_passes, int32_t *final_cache, int32_t *passes,
                      int64_t *changed, int32_t *caches)
{
    int32_t *prev = (int32_t *)malloc(sizeof(int32_t) * (size_t)(T + 1));
    int32_t *next = (int32_t *)malloc(sizeof(int32_t) * (size_t)(T + 1));
    if (!prev || !next) { free(prev); free(next); return -1; }
    for (int64_t t = 0; t < T; ++t) prev[t] = init_cache ? init_cache[t] : LOST;
    int rc = 1;
    int32_t k;
    for (k = 1; k <= max_passes; ++k) {
        pass(ctx, prev, next);
        if (caches) memcpy(caches + (int64_t)(k - 1) * T, next, sizeof(int32_t) * (size_t)T);
        int64_t nch = 0;
        for (int64_t t = 0; t < T; ++t) nch += next[t] != prev[t];
        if (changed) changed[k - 1] = nch;
        int32_t *tmp = prev; prev = next; next = tmp;
        if (nch == 0) { rc = 0; break; }
    }
    if (k > max_passes) k = max_passes;
    *passes = k;
    memcpy(final_cache, prev, sizeof(int32_t) * (size_t)T);
    free(prev);
    free(next);
    return rc;
}

/* ------------------------------------------------------------------------------------
 * Policy evaluated at the states induced by a given action sequence.
 * choice[t] = pi(s_t) where s_t follows from actions[0..t-1]; z1/z2 as in policy();
 * n_feasible[t] = |{w : x[w] > 0}|.  Any pointer but actions/choice may be NULL.
 * Returns -2 if a given action is infeasible at its state (it cannot come from pi).
 * ---------------------------------------------------------------------------------- */
int orc_eval_at_range(const orc_problem *P, const int32_t *actions, int64_t lo, int64_t hi,
                      int32_t *choice, double *z1, double *z2, int32_t *n_feasible);

int orc_eval_at(const orc_problem *P, const int32_t *actions, int32_t *choice, double *z1,
                double *z2, int32_t *n_feasible)
{
    return orc_eval_at_range(P, actions, 0, P->T, choice, z1, z2, n_feasible);
}

/* The same, with the policy evaluated only at steps lo <= t < hi (outputs written there
 * only): the steps before lo just apply their given actions, so disjoint windows can be
 * evaluated independently. */
int orc_eval_at_range(const orc_problem *P, const int32_t *actions, int64_t lo, int64_t hi,
                      int32_t *choice, double *z1, double *z2, int32_t *n_feasible)
{
    if (check_problem(P) || lo < 0 || hi > P->T || lo > hi) return -1;
    const int N = P->N;
    mlp64 m = {0};
    if (P->params && mlp_load(&m, P)) return -1;
    int32_t *x = (int32_t *)malloc(sizeof(int32_t) * (size_t)P->K * N);
    if (!x) { mlp_free(&m); return -1; }
    memcpy(x, P->x0, sizeof(int32_t) * (size_t)P->K * N);
    int rc = 0;
    for (int64_t t = 0; t < hi; ++t) {
        int32_t *xk = x + (int64_t)P->sku[t] * N;
        if (t < lo) { /* replay only */
            int32_t a = actions[t];
            if (a != LOST && (a < 0 || a >= N || xk[a] <= 0)) { rc = -2; break; }
            transition(xk, a, P->qty[t]);
            continue;
        }
        double a1 = -INFINITY, a2 = -INFINITY;
        choice[t] = policy(P, &m, t, xk, &a1, &a2);
        if (z1) z1[t] = a1;
        if (z2) z2[t] = a2;
        if (n_feasible) {
            int32_t c = 0;
            for (int w = 0; w < N; ++w) c += xk[w] > 0;
            n_feasible[t] = c;
        }
        int32_t a = actions[t];
        if (a != LOST && (a < 0 || a >= N || xk[a] <= 0)) { rc = -2; break; }
        transition(xk, a, P->qty[t]);
    }
    free(x);
    mlp_free(&m);
    return rc;
}

/* ------------------------------------------------------------------------------------
 * Algorithm 1 by brute force, for any assignment worker[t] in [0, n_workers) of steps to
 * processes: in a pass every process has its own view of the whole horizon (its own
 * steps decided fresh, everyone else's taken from the previous cache), and the new
 * cache collects each step's decision from the view of the process that owns it.
 * init_cache may be NULL (alpha^0 = lost sale everywhere); caches, return value and
 * passes as run_passes.  O(P*T*N) per pass: tiny instances only.
 * ---------------------------------------------------------------------------------- */
typedef struct {
    const orc_problem *P;
    const mlp64 *m;
    const int64_t *worker;
    int64_t n_workers;
    int32_t *x;
} alg1_ctx;

static void alg1_pass(void *vctx, const int32_t *prev, int32_t *next)
{
    const alg1_ctx *c = (const alg1_ctx *)vctx;
    for (int64_t proc = 0; proc < c->n_workers; ++proc)
        process_view(c->P, c->m, c->worker, proc, prev, next, c->x, NULL, NULL, NULL);
}

int orc_alg1(const orc_problem *P, const int64_t *worker, int64_t n_workers,
             const int32_t *init_cache, int32_t max_passes, int32_t *final_cache,
             int32_t *passes, int32_t *caches)
{
    if (check_problem(P) || n_workers <= 0 || max_passes <= 0) return -1;
    for (int64_t t = 0; t < P->T; ++t)
        if (worker[t] < 0 || worker[t] >= n_workers) return -1;
    mlp64 m = {0};
    if (P->params && mlp_load(&m, P)) return -1;
    int32_t *x = (int32_t *)malloc(sizeof(int32_t) * (size_t)P->K * P->N);
    if (!x) { mlp_free(&m); return -1; }
    alg1_ctx ctx = {P, &m, worker, n_workers, x};
    const int rc = run_passes(alg1_pass, &ctx, P->T, init_cache, max_passes, final_cache,
                              passes, NULL, caches);
    free(x);
    mlp_free(&m);
    return rc;
}

/* ------------------------------------------------------------------------------------
 * The same passes, per SKU.  Orders of SKU k in time order form its segment; a run is
 * a maximal stretch of the segment owned by one process.  Per pass and per segment,
 * runs are visited in order:
 *   entry state = max(0, x0[k] - E - D), E = cached consumption (sum of q over earlier
 *   runs' orders sent to each warehouse under alpha^{k-1}), D = the run's process's own
 *   correction: over its earlier runs of this segment, q at the warehouse it chose in
 *   this pass minus q at the cached warehouse (0 when the process owns one run);
 *   the run is walked with the process's own decisions.
 * changed (nullable): number of steps with alpha^k != alpha^{k-1}, per pass.
 * ---------------------------------------------------------------------------------- */
int orc_picard_runs(const orc_problem *P, const int64_t *worker, const int32_t *init_cache,
                    int32_t max_passes, int32_t *final_cache, int32_t *passes,
                    int64_t *changed, int32_t *caches)
{
    if (check_problem(P) || max_passes <= 0) return -1;
    const int N = P->N, K = P->K;
    const int64_t T = P->T;
    mlp64 m = {0};
    if (P->params && mlp_load(&m, P)) return -1;
    /* stable counting sort of steps by SKU */
    int64_t *start = (int64_t *)calloc((size_t)K + 1, sizeof(int64_t));
    int64_t *fill = (int64_t *)calloc((size_t)K + 1, sizeof(int64_t));
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(T + 1));
    int32_t *prev = (int32_t *)malloc(sizeof(int32_t) * (size_t)(T + 1));
    int32_t *next = (int32_t *)malloc(sizeof(int32_t) * (size_t)(T + 1));
    int64_t *E = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    int64_t *D = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    int32_t *x = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int rc = 0;
    if (!start || !fill || !pos || !prev || !next || !E || !D || !x) { rc = -1; goto done; }
    for (int64_t t = 0; t < T; ++t) start[P->sku[t] + 1]++;
    for (int k = 0; k < K; ++k) start[k + 1] += start[k];
    for (int64_t t = 0; t < T; ++t) {
        int s = P->sku[t];
        pos[start[s] + fill[s]++] = t;
    }
    for (int64_t t = 0; t < T; ++t) prev[t] = init_cache ? init_cache[t] : LOST;
    rc = 1;
    int32_t k;
    for (k = 1; k <= max_passes; ++k) {
        for (int s = 0; s < K; ++s) {
            for (int w = 0; w < N; ++w) E[w] = 0;
            const int32_t *x0k = P->x0 + (int64_t)s * N;
            int64_t i = start[s];
            while (i < start[s + 1]) {
                int64_t j = i;
                while (j < start[s + 1] && worker[pos[j]] == worker[pos[i]]) ++j;
                /* the process's own earlier orders of this segment: fresh minus cached */
                for (int w = 0; w < N; ++w) D[w] = 0;
                for (int64_t p = start[s]; p < i; ++p) {
                    int64_t t = pos[p];
                    if (worker[t] != worker[pos[i]]) continue;
                    if (next[t] != LOST) D[next[t]] += P->qty[t];
                    if (prev[t] != LOST) D[prev[t]] -= P->qty[t];
                }
                for (int w = 0; w < N; ++w) {
                    int64_t v = (int64_t)x0k[w] - E[w] - D[w];
                    x[w] = v > 0 ? (int32_t)v : 0;
                }
                for (int64_t p = i; p < j; ++p) {
                    int64_t t = pos[p];
                    int32_t a = policy(P, &m, t, x, NULL, NULL);
                    next[t] = a;
                    transition(x, a, P->qty[t]);
                }
                for (int64_t p = i; p < j; ++p) {
                    int64_t t = pos[p];
                    if (prev[t] != LOST) E[prev[t]] += P->qty[t];
                }
                i = j;
            }
        }
        int64_t nchg = 0;
        for (int64_t t = 0; t < T; ++t) nchg += next[t] != prev[t];
        if (changed) changed[k - 1] = nchg;
        if (caches) memcpy(caches + (int64_t)(k - 1) * T, next, sizeof(int32_t) * (size_t)T);
        int32_t *tmp = prev; prev = next; next = tmp;
        if (nchg == 0) { rc = 0; break; }
    }
    if (k > max_passes) k = max_passes;
    *passes = k;
    memcpy(final_cache, prev, sizeof(int32_t) * (size_t)T);
done:
    free(start); free(fill); free(pos); free(prev); free(next); free(E); free(D); free(x);
    mlp_free(&m);
    return rc;
}

/* ------------------------------------------------------------------------------------
 * REINFORCE surrogate and gradient, FP64, at fixed actions.
 *   L = sum_t A_t log pi(a_t | s_t),  pi(. | s) = softmax over feasible w of s_w
 * (the Gumbel-max rule samples exactly from this softmax).  Steps with no feasible
 * warehouse contribute 0 (then a_t must be the lost sale).  logp[t] (nullable) receives
 * log pi(a_t | s_t); grad (nullable) the gradient in the parameter-pack layout.
 * Returns -2 when an action is not in the feasible set of its state.
 * ---------------------------------------------------------------------------------- */
int orc_reinforce_range(const orc_problem *P, const int32_t *actions, const double *adv,
                        int64_t lo, int64_t hi, double *logp, double *grad, double *objective);

int orc_reinforce(const orc_problem *P, const int32_t *actions, const double *adv,
                  double *logp, double *grad, double *objective)
{
    return orc_reinforce_range(P, actions, adv, 0, P->T, logp, grad, objective);
}

/* The terms of steps lo <= t < hi only (the steps before lo just apply their actions):
 * the surrogate and its gradient are sums over steps, so the sum over disjoint windows
 * covering [0, T) is the whole. */
int orc_reinforce_range(const orc_problem *P, const int32_t *actions, const double *adv,
                        int64_t lo, int64_t hi, double *logp, double *grad, double *objective)
{
    if (check_problem(P) || !P->params || lo < 0 || hi > P->T || lo > hi) return -1;
    const int N = P->N, R = P->R;
    mlp64 m = {0};
    if (mlp_load(&m, P)) return -1;
    const int H = m.H;
    if (H > 1024) { mlp_free(&m); return -1; }
    int64_t np = param_count(R, H, m.L);
    double *g = grad ? grad : NULL;
    if (g) memset(g, 0, sizeof(double) * (size_t)np);
    double *gE = g, *gW1 = g ? g + (int64_t)R * 16 : NULL;
    double *gb1 = gW1 ? gW1 + (int64_t)H * 18 : NULL;
    double *gW2 = NULL, *gb2 = NULL, *gw3, *gb3;
    if (m.L == 2 && g) { gW2 = gb1 + H; gb2 = gW2 + (int64_t)H * H; gw3 = gb2 + H; }
    else gw3 = gb1 ? gb1 + H : NULL;
    gb3 = gw3 ? gw3 + H : NULL;

    int32_t *x = (int32_t *)malloc(sizeof(int32_t) * (size_t)P->K * N);
    double *s = (double *)malloc(sizeof(double) * (size_t)N);
    double *F = (double *)malloc(sizeof(double) * (size_t)N * 18);
    double *PRE1 = (double *)malloc(sizeof(double) * (size_t)N * H);
    double *H1 = (double *)malloc(sizeof(double) * (size_t)N * H);
    double *PRE2 = (double *)malloc(sizeof(double) * (size_t)N * H);
    double *H2 = (double *)malloc(sizeof(double) * (size_t)N * H);
    double *dh = (double *)malloc(sizeof(double) * (size_t)H);
    double *dp2 = (double *)malloc(sizeof(double) * (size_t)H);
    double *dp1 = (double *)malloc(sizeof(double) * (size_t)H);
    int rc = 0;
    if (!x || !s || !F || !PRE1 || !H1 || !PRE2 || !H2 || !dh || !dp2 || !dp1) { rc = -1; goto out; }
    memcpy(x, P->x0, sizeof(int32_t) * (size_t)P->K * N);
    double L = 0.0;
    for (int64_t t = 0; t < hi; ++t) {
        int32_t *xk = x + (int64_t)P->sku[t] * N;
        const int r = P->region[t];
        const int32_t a = actions[t];
        if (t < lo) { /* replay only */
            if (a != LOST && (a < 0 || a >= N || xk[a] <= 0)) { rc = -2; break; }
            transition(xk, a, P->qty[t]);
            continue;
        }
        int nf = 0;
        for (int w = 0; w < N; ++w) nf += xk[w] > 0;
        if (nf == 0) {
            if (a != LOST) { rc = -2; break; }
            if (logp) logp[t] = 0.0;
            continue;
        }
        if (a < 0 || a >= N || xk[a] <= 0) { rc = -2; break; }
        double mx = -INFINITY;
        for (int w = 0; w < N; ++w) {
            if (xk[w] <= 0) continue;
            s[w] = mlp_forward(&m, (double)P->cost[w * R + r], (double)xk[w], r, F + w * 18,
                               PRE1 + (int64_t)w * H, H1 + (int64_t)w * H,
                               PRE2 + (int64_t)w * H, H2 + (int64_t)w * H);
            if (s[w] > mx) mx = s[w];
        }
        double se = 0.0;
        for (int w = 0; w < N; ++w)
            if (xk[w] > 0) se += exp(s[w] - mx);
        const double lse = mx + log(se);
        const double lp = s[a] - lse;
        if (logp) logp[t] = lp;
        L += adv[t] * lp;
        if (g) {
            for (int w = 0; w < N; ++w) {
                if (xk[w] <= 0) continue;
                const double p = exp(s[w] - lse);
                const double ds = adv[t] * ((w == a ? 1.0 : 0.0) - p);
                const double *h1 = H1 + (int64_t)w * H, *h2 = H2 + (int64_t)w * H;
                const double *pre1 = PRE1 + (int64_t)w * H, *pre2 = PRE2 + (int64_t)w * H;
                const double *hl = m.L == 2 ? h2 : h1;
                *gb3 += ds;
                for (int j = 0; j < H; ++j) { gw3[j] += ds * hl[j]; dh[j] = ds * m.w3[j]; }
                if (m.L == 2) {
                    for (int j = 0; j < H; ++j) dp2[j] = pre2[j] > 0.0 ? dh[j] : 0.0;
                    for (int j = 0; j < H; ++j) {
                        gb2[j] += dp2[j];
                        for (int i = 0; i < H; ++i) gW2[j * H + i] += dp2[j] * h1[i];
                    }
                    for (int i = 0; i < H; ++i) {
                        double acc = 0.0;
                        for (int j = 0; j < H; ++j) acc += m.W2[j * H + i] * dp2[j];
                        dh[i] = acc;
                    }
                }
                for (int j = 0; j < H; ++j) dp1[j] = pre1[j] > 0.0 ? dh[j] : 0.0;
                const double *f = F + w * 18;
                for (int j = 0; j < H; ++j) {
                    gb1[j] += dp1[j];
                    for (int i = 0; i < 18; ++i) gW1[j * 18 + i] += dp1[j] * f[i];
                }
                for (int i = 0; i < 16; ++i) {
                    double acc = 0.0;
                    for (int j = 0; j < H; ++j) acc += m.W1[j * 18 + 2 + i] * dp1[j];
                    gE[r * 16 + i] += acc;
                }
            }
        }
        transition(xk, a, P->qty[t]);
    }
    if (objective) *objective = L;
out:
    free(x); free(s); free(F); free(PRE1); free(H1); free(PRE2); free(H2);
    free(dh); free(dp2); free(dp1);
    mlp_free(&m);
    return rc;
}

/* The policy pi(s_t, w_t) at given states: for i < n, order ts[i] of the trajectory
 * (its region and noise) with its SKU's inventory row x_rows[i * N .. i * N + N) (the other
 * SKUs' rows do not enter the decision).  choice[i], and z1[i] >= z2[i] the two largest
 * perturbed scores among warehouses with stock (nullable).  Only the orders' regions,
 * the costs, the parameters and the noise key of P are read. */
int orc_policy_at(const orc_problem *P, int64_t n, const int64_t *ts, const int32_t *x_rows,
                  int32_t *choice, double *z1, double *z2)
{
    if (P->N <= 0 || P->R <= 0 || n < 0) return -1;
    mlp64 m = {0};
    if (P->params && mlp_load(&m, P)) return -1;
    int rc = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t t = ts[i];
        if (t < 0 || t >= P->T || P->region[t] < 0 || P->region[t] >= P->R) { rc = -1; break; }
        double a1 = -INFINITY, a2 = -INFINITY;
        choice[i] = policy(P, &m, t, x_rows + i * (int64_t)P->N, &a1, &a2);
        if (z1) z1[i] = a1;
        if (z2) z2[i] = a2;
    }
    mlp_free(&m);
    return rc;
}

/* Raw (noise-free) scores of every warehouse for region r at inventory row x. */
int orc_mlp_scores(const orc_problem *P, int32_t r, const int32_t *x, double *s)
{
    if (!P->params || r < 0 || r >= P->R) return -1;
    mlp64 m = {0};
    if (mlp_load(&m, P)) return -1;
    for (int w = 0; w < P->N; ++w)
        s[w] = mlp_forward(&m, (double)P->cost[w * P->R + r], (double)x[w], r, NULL, NULL,
                           NULL, NULL, NULL);
    mlp_free(&m);
    return 0;
}

/* ====================================================================================
 * Node capacity (Section 3, the FO model in full): the state is (x_t, c_t); an order of
 * SKU i may go to node j only if c_{t,j} > 0 and x_{t,i,j} > 0; shipping it lowers
 * c_{t,j} and x_{t,i,j} by one.  The paper's transition is unit demand, so every order
 * here must have q = 1.  Policy: greedy (least cost[j][region] among nodes with both
 * capacity and stock, lowest index on ties; lost sale iff none), as in Section 3.1, the
 * capacity-dependent policy of the appendix's ablation, or a bid-price policy (greedy_cap).
 * cap0[N] >= 0 is c_1.
 * ==================================================================================== */
/* The policy with capacity: the greedy policy (gnum = 0, no bid prices), the
 * capacity-dependent policy of the appendix's ablation (gnum > 0), or a bid-price policy
 * (bid_inv and/or bid_cap given, gnum = 0). */
typedef struct {
    int32_t gnum, gden, glow;
    const int32_t *bid_inv; /* nullable [K][N]: price of a unit of SKU k's stock at node w */
    const int32_t *bid_cap; /* nullable [N]: price of a unit of node w's capacity */
} orc_cap_policy;

static int check_cap(const orc_problem *P, const int32_t *cap0, const orc_cap_policy *pol)
{
    if (check_problem(P) || P->params || !pol) return -1;
    const int32_t gnum = pol->gnum, gden = pol->gden, glow = pol->glow;
    if (gnum < 0 || gden < 1 || gnum > 1000 || gden > 1000 || glow < 0) return -1;
    if ((pol->bid_inv || pol->bid_cap) && gnum != 0) return -1;
    for (int64_t t = 0; t < P->T; ++t)
        if (P->qty[t] != 1) return -1;
    for (int w = 0; w < P->N; ++w)
        if (cap0[w] < 0) return -1;
    return 0;
}

/* The policy with capacity, at state (x row of the order's SKU, capacities c).
 * gnum = 0: greedy, the feasible node of least cost[w][region], lowest index on ties.
 * gnum > 0: the capacity-dependent policy of the appendix's ablation, gamma = gnum/gden:
 * node w's rank in the region's (cost, index) order, rank_r(w) in 0..N-1, is worsened by
 * a shadow price gamma (N-1) p_w, in one of two readings:
 *   glow = 0: p_w = 1 - c_w / M, M the largest remaining capacity of any node, so the
 *     node with the most capacity left can rise up to gamma (N-1) places;
 *   glow > 0: p_w = max(0, glow - c_w) / glow, only nodes with less than glow capacity
 *     left pay a price, rising to gamma (N-1) as they empty.
 * Compared exactly, with M = glow in the second reading, as
 *   gden rank_r(w) M + gnum (N-1) M p_w   (both sides times gden M > 0),
 * least first, lowest index on ties; lost sale iff no node is feasible. */
static int32_t rank_in_region(const orc_problem *P, int r, int w)
{
    const int R = P->R;
    const int32_t cw = P->cost[w * R + r];
    int32_t k = 0;
    for (int v = 0; v < P->N; ++v) {
        const int32_t cv = P->cost[v * R + r];
        if (cv < cw || (cv == cw && v < w)) ++k;
    }
    return k;
}

/* rank_in_region for every (region, node), once per call: [R][N]; NULL when gnum = 0. */
static int32_t *rank_table(const orc_problem *P, int32_t gnum)
{
    if (gnum == 0) return NULL;
    int32_t *rk = (int32_t *)malloc(sizeof(int32_t) * (size_t)P->R * P->N);
    if (!rk) return NULL;
    for (int r = 0; r < P->R; ++r)
        for (int w = 0; w < P->N; ++w) rk[(int64_t)r * P->N + w] = rank_in_region(P, r, w);
    return rk;
}

static int32_t greedy_cap(const orc_problem *P, int64_t t, const int32_t *x, const int32_t *c,
                          const orc_cap_policy *pol, const int32_t *rk)
{
    const int R = P->R, r = P->region[t];
    const int32_t gnum = pol->gnum, gden = pol->gden, glow = pol->glow;
    int32_t best = LOST;
    if (pol->bid_inv || pol->bid_cap) {
        /* bid prices: the least cost plus the prices of the unit of stock and of capacity
         * the order would use (the dual policy of Section 4.2 with fixed prices) */
        const int32_t *bi = pol->bid_inv ? pol->bid_inv + (int64_t)P->sku[t] * P->N : NULL;
        int64_t best_s = 0;
        for (int w = 0; w < P->N; ++w) {
            if (x[w] <= 0 || c[w] <= 0) continue;
            const int64_t sc = (int64_t)P->cost[w * R + r] + (bi ? bi[w] : 0) +
                               (pol->bid_cap ? pol->bid_cap[w] : 0);
            if (best == LOST || sc < best_s) { best = w; best_s = sc; }
        }
        return best;
    }
    if (gnum == 0) {
        int32_t best_cost = 0;
        for (int w = 0; w < P->N; ++w) {
            if (x[w] <= 0 || c[w] <= 0) continue;
            const int32_t cw = P->cost[w * R + r];
            if (best == LOST || cw < best_cost) { best = w; best_cost = cw; }
        }
        return best;
    }
    int64_t M = glow;
    if (glow == 0)
        for (int w = 0; w < P->N; ++w)
            if (c[w] > M) M = c[w];
    int64_t best_s = 0;
    for (int w = 0; w < P->N; ++w) {
        if (x[w] <= 0 || c[w] <= 0) continue;
        const int64_t price = glow == 0 ? M - c[w] : (c[w] < glow ? (int64_t)glow - c[w] : 0);
        const int64_t sc = (int64_t)gden * rk[(int64_t)r * P->N + w] * M +
                           (int64_t)gnum * (P->N - 1) * price;
        if (best == LOST || sc < best_s) { best = w; best_s = sc; }
    }
    return best;
}

/* f with capacity: one unit leaves both counters when the action is a node. */
static void transition_cap(int32_t *x, int32_t *c, int32_t a)
{
    if (a == LOST) return;
    x[a] -= 1;
    c[a] -= 1;
}

/* One process's view of the horizon with capacity: as process_view, with the state
 * (x, c) starting at (x0, cap0); a given action is replaced by the lost sale when its
 * node has no stock of the SKU or no capacity left in the view.  x: K*N scratch, c: N. */
static void process_view_cap(const orc_problem *P, const int32_t *cap0,
                             const orc_cap_policy *pol, const int32_t *rk, const int64_t *owner,
                             int64_t self, const int32_t *given, int32_t *decided, int32_t *x,
                             int32_t *c)
{
    const int N = P->N;
    memcpy(x, P->x0, sizeof(int32_t) * (size_t)P->K * N); /* every view starts at s_1 */
    memcpy(c, cap0, sizeof(int32_t) * (size_t)N);
    for (int64_t t = 0; t < P->T; ++t) {
        int32_t *xk = x + (int64_t)P->sku[t] * N;
        int32_t a;
        if (!owner || owner[t] == self) {
            a = greedy_cap(P, t, xk, c, pol, rk);
            decided[t] = a;
        } else {
            a = given[t];
            if (a != LOST && (a < 0 || a >= N || xk[a] <= 0 || c[a] <= 0)) a = LOST;
        }
        transition_cap(xk, c, a);
    }
}

/* Serial rollout with capacity (the answer Picard must reach): the view of a process
 * that owns every order. */
int orc_serial_cap(const orc_problem *P, const int32_t *cap0, const orc_cap_policy *pol,
                   int32_t *actions, int32_t *final_inv, int32_t *final_cap)
{
    if (check_cap(P, cap0, pol)) return -1;
    const int N = P->N;
    int32_t *rk = rank_table(P, pol->gnum);
    if (pol->gnum && !rk) return -1;
    int32_t *x = (int32_t *)malloc(sizeof(int32_t) * (size_t)P->K * N);
    int32_t *c = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    if (!x || !c) { free(x); free(c); free(rk); return -1; }
    process_view_cap(P, cap0, pol, rk, NULL, 0, NULL, actions, x, c);
    if (final_inv) memcpy(final_inv, x, sizeof(int32_t) * (size_t)P->K * N);
    if (final_cap) memcpy(final_cap, c, sizeof(int32_t) * (size_t)N);
    free(x);
    free(c);
    free(rk);
    return 0;
}

/* Algorithm 1 with capacity by brute force: as orc_alg1, every process's view carrying
 * its own (x, c).  O(P*T*N) per pass: tiny instances only. */
typedef struct {
    const orc_problem *P;
    const int32_t *cap0, *rk;
    const orc_cap_policy *pol;
    const int64_t *worker;
    int64_t n_workers;
    int32_t *x, *c;
} alg1_cap_ctx;

static void alg1_cap_pass(void *vctx, const int32_t *prev, int32_t *next)
{
    const alg1_cap_ctx *q = (const alg1_cap_ctx *)vctx;
    for (int64_t proc = 0; proc < q->n_workers; ++proc)
        process_view_cap(q->P, q->cap0, q->pol, q->rk, q->worker, proc, prev, next, q->x,
                         q->c);
}

int orc_alg1_cap(const orc_problem *P, const int32_t *cap0, const orc_cap_policy *pol,
                 const int64_t *worker, int64_t n_workers, const int32_t *init_cache,
                 int32_t max_passes, int32_t *final_cache, int32_t *passes, int32_t *caches)
{
    if (check_cap(P, cap0, pol) || n_workers <= 0 || max_passes <= 0) return -1;
    const int N = P->N;
    for (int64_t t = 0; t < P->T; ++t)
        if (worker[t] < 0 || worker[t] >= n_workers) return -1;
    int32_t *rk = rank_table(P, pol->gnum);
    if (pol->gnum && !rk) return -1;
    int32_t *x = (int32_t *)malloc(sizeof(int32_t) * (size_t)P->K * N);
    int32_t *c = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    if (!x || !c) { free(x); free(c); free(rk); return -1; }
    alg1_cap_ctx ctx = {P, cap0, rk, pol, worker, n_workers, x, c};
    const int rc = run_passes(alg1_cap_pass, &ctx, P->T, init_cache, max_passes, final_cache,
                              passes, NULL, caches);
    free(x); free(c); free(rk);
    return rc;
}

/* The same passes for the partition into time blocks: process m owns the B consecutive
 * steps [mB, (m+1)B).  Every process replays the cached actions of all steps before
 * its block, and nothing after its block reaches its decisions, so each process starts
 * its block from one shared state: the replay of alpha^{k-1} (infeasible cached actions
 * replaced by lost sales) up to the block.  One pass is then a single replay in time
 * order; at the start of block m, process m walks its B steps with fresh decisions on a
 * private copy of the shared state (the rows of the SKUs it meets, copied on first use,
 * and the capacities), after which the replay applies the block's cached actions.
 * O(T*N) per pass.  changed (nullable) receives |{t : alpha^k_t != alpha^{k-1}_t}| per
 * pass.  Other arguments and the return value as orc_alg1. */
typedef struct {
    const orc_problem *P;
    const int32_t *cap0, *rk;
    const orc_cap_policy *pol;
    int64_t B;
    int32_t *x, *xp, *c, *cp; /* shared replay, private rows, shared and private capacities */
    int64_t *stamp;           /* block that last copied a SKU's row into xp */
} blocks_cap_ctx;

static void timeblocks_cap_pass(void *vctx, const int32_t *prev, int32_t *next)
{
    const blocks_cap_ctx *q = (const blocks_cap_ctx *)vctx;
    const orc_problem *P = q->P;
    const int N = P->N;
    const int64_t T = P->T, B = q->B;
    int32_t *x = q->x, *xp = q->xp, *c = q->c, *cp = q->cp;
    memcpy(x, P->x0, sizeof(int32_t) * (size_t)P->K * N);
    memcpy(c, q->cap0, sizeof(int32_t) * (size_t)N);
    for (int64_t i = 0; i < P->K; ++i) q->stamp[i] = -1;
    for (int64_t m = 0; m * B < T; ++m) {
        const int64_t lo = m * B, hi = lo + B < T ? lo + B : T;
        /* process m: fresh decisions from the shared state */
        memcpy(cp, c, sizeof(int32_t) * (size_t)N);
        for (int64_t t = lo; t < hi; ++t) {
            const int64_t s = P->sku[t];
            int32_t *xk = xp + s * N;
            if (q->stamp[s] != m) {
                memcpy(xk, x + s * N, sizeof(int32_t) * (size_t)N);
                q->stamp[s] = m;
            }
            const int32_t a = greedy_cap(P, t, xk, cp, q->pol, q->rk);
            transition_cap(xk, cp, a);
            next[t] = a;
        }
        /* the shared replay applies the block's cached actions */
        for (int64_t t = lo; t < hi; ++t) {
            int32_t *xk = x + (int64_t)P->sku[t] * N;
            int32_t a = prev[t];
            if (a != LOST && (a < 0 || a >= N || xk[a] <= 0 || c[a] <= 0)) a = LOST;
            transition_cap(xk, c, a);
        }
    }
}

int orc_picard_timeblocks_cap(const orc_problem *P, const int32_t *cap0,
                              const orc_cap_policy *pol, int64_t B, const int32_t *init_cache,
                              int32_t max_passes, int32_t *final_cache, int32_t *passes,
                              int64_t *changed, int32_t *caches)
{
    if (check_cap(P, cap0, pol) || B <= 0 || max_passes <= 0) return -1;
    const int N = P->N, K = P->K;
    int32_t *rk = rank_table(P, pol->gnum);
    if (pol->gnum && !rk) return -1;
    const int64_t KN = (int64_t)K * N;
    int32_t *x = (int32_t *)malloc(sizeof(int32_t) * (size_t)KN);
    int32_t *xp = (int32_t *)malloc(sizeof(int32_t) * (size_t)KN);
    int64_t *stamp = (int64_t *)malloc(sizeof(int64_t) * (size_t)K);
    int32_t *c = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int32_t *cp = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int rc = -1;
    if (x && xp && stamp && c && cp) {
        blocks_cap_ctx ctx = {P, cap0, rk, pol, B, x, xp, c, cp, stamp};
        rc = run_passes(timeblocks_cap_pass, &ctx, P->T, init_cache, max_passes, final_cache,
                        passes, changed, caches);
    }
    free(x); free(xp); free(stamp); free(c); free(cp); free(rk);
    return rc;
}

/*
 * libpicard: Picard-iteration policy simulation for the fulfillment problem on MI355X.
 *
 * The problem (Section 2, problem statement): given an initial state s_1, a horizon T and
 * disturbances w_1..w_T, produce the actions a_t = pi(s_t, w_t) of the serial rollout
 * s_{t+1} = f(s_t, a_t, w_t).  Here the state is the inventory x[k][w] of K SKUs at N
 * warehouses, an order (disturbance) carries a SKU, a region and a quantity, and the
 * transition (Section 3, FO model, without node capacity) ships min(q, x[k][a]) from the
 * chosen warehouse a; the always-feasible action a^phi is the lost sale PK_LOST.
 *
 * pk_picard_simulate computes that rollout with Algorithm 1 (the Picard iteration):
 * steps are split among processes, every step keeps a cached action, each pass
 * rebuilds every process's state from the cache, re-evaluates the policy on all
 * process-owned steps at once and rewrites the cache, and the iteration stops at the
 * first pass that changes nothing, whose cache equals the serial rollout
 * (Proposition 2.1).
 *
 * Conventions shared by every entry point
 *   - Array pointers are DEVICE pointers (memory of the current HIP device) unless
 *     marked HOST.  The caller owns every buffer; the library only borrows them for the
 *     duration of the call and never frees or keeps them.
 *   - Work is enqueued on `stream` (0 = the null stream).  Calls that iterate to
 *     convergence block the calling thread until the result is final.
 *   - Orders of a batch of independent trajectories are concatenated: trajectory b owns
 *     orders [traj_offsets[b], traj_offsets[b+1]) in time order.
 *   - Scratch memory is the caller's `ws` buffer of `ws_bytes` bytes; its size comes from
 *     pk_workspace_size for the same problem, policy and options.
 *   - No exception or abort crosses this interface.  On any status other than PK_OK,
 *     pk_last_error() returns a message (thread-local, valid until the next call).
 *   - Host-side shape checks always run.  Device-side range checks of the inputs
 *     (SKU, region, quantity, initial inventory, initial cache) run when
 *     pk_picard_opts.validate (or the validate argument) is nonzero.
 */
#ifndef PICARD_H
#define PICARD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PK_OK = 0,
    PK_ERR_INVALID_ARG = -1,   /* a pointer, size or option is invalid, or validate found
                                  an out-of-range input value */
    PK_ERR_SHAPE = -2,         /* dimensions inconsistent or beyond the supported limits */
    PK_ERR_HIP = -3,           /* a HIP runtime call failed */
    PK_ERR_NOT_CONVERGED = -4, /* max_passes reached; outputs hold the last cache */
    PK_ERR_WORKSPACE = -5,     /* ws is NULL or smaller than pk_workspace_size */
    PK_ERR_UNSUPPORTED = -6,   /* a valid request this build does not implement */
    PK_ERR_INTERNAL = -7       /* a device-side consistency check failed (a defect of the
                                  library, not of the input); outputs are undefined */
} pk_status;

#define PK_LOST (-1) /* the lost sale a^phi: no warehouse ships the order */

/* Limits of this build (checked on the host, PK_ERR_SHAPE beyond them). */
#define PK_MAX_WAREHOUSES 1024
#define PK_MAX_REGIONS 4096

/* The inputs s_1 and {w_t} of the problem statement (Section 2), instantiated for the
 * FO model of Section 3 (products -> SKUs, nodes -> warehouses, reward r_w(w_t) ->
 * -cost[w][region_t]). */
typedef struct pk_problem {
    int32_t n_warehouses;          /* N >= 1 */
    int32_t n_skus;                /* K >= 1 */
    int32_t n_regions;             /* R >= 1 */
    int32_t n_traj;                /* trajectories in the batch, >= 1 */
    const int64_t *traj_offsets;   /* HOST [n_traj+1], nondecreasing, traj_offsets[0] = 0,
                                      total orders traj_offsets[n_traj] < 2^31 */
    const int32_t *sku;            /* [total] in [0, K) */
    const int32_t *region;         /* [total] in [0, R) */
    const int32_t *qty;            /* [total] >= 1 */
    const int32_t *init_inv;       /* [n_traj][K][N] x0 >= 0 */
    const int32_t *cost;           /* [n_traj][N][R] order cost of warehouse w for region r */
    uint64_t rng_seed;             /* Philox4x32-10 key of the learned policy's noise */
} pk_problem;

typedef enum { PK_POLICY_GREEDY = 0, PK_POLICY_MLP = 1 } pk_policy_kind;

/* The policy pi.
 * GREEDY (Section 3.1 greedy policy, inventory as the constraint): the warehouse with
 *   stock (x > 0) of least cost[w][region], lowest index on ties; PK_LOST iff none.
 * MLP (learned softmax policy, Section 4.2 trains a policy by policy gradient): score
 *   s_w = mlp(cost[w][r], log1p(x[k][w]), E[r]) with two (or one) ReLU hidden layers
 *   of width `hidden`; the action is argmax over warehouses with stock of
 *   s_w + G(t, traj, w), G a Gumbel variate from Philox4x32-10 (key rng_seed, counter
 *   (t, traj, w >> 2, 0), output word w & 3, U = ((u >> 9) + 0.5) 2^-23,
 *   G = -log(-log U)), lowest index on exact ties; this samples softmax(s) over the
 *   warehouses with stock.  The noise is part of the disturbance (Section 2).
 * params (MLP only; DEVICE, float32, caller-owned), flat pack:
 *   E[R][16] | W1[hidden][18] | b1[hidden] | (W2[hidden][hidden] | b2[hidden]) | w3[hidden] | b3
 *   feature order [cost, log1p(inventory), E[region][0..15]]; W2/b2 absent with one layer. */
typedef struct pk_policy {
    int32_t kind;            /* pk_policy_kind */
    int32_t n_hidden_layers; /* MLP: 1 or 2 */
    int32_t hidden;          /* MLP: 64 */
    int32_t emb_dim;         /* MLP: 16 */
    const float *params;     /* MLP: device parameter pack; ignored by GREEDY */
} pk_policy;

/* Options of the Picard iteration (Algorithm 1 and Appendix A.3's restart rule). */
typedef struct pk_picard_opts {
    int32_t block_len;    /* Partition: the batch's orders sorted by (trajectory, SKU),
                             ties in time order, are cut into blocks of block_len
                             consecutive positions; block m is process m.  1 gives every
                             step its own process; a block at least as long as every
                             SKU's order list is a product partition (Section 3).
                             0 = autotuned. */
    int32_t max_passes;   /* cap on passes; 0 = (longest horizon) + 1, the bound of
                             Proposition 2.1 plus the confirming pass */
    int32_t use_frontier; /* 1: skip steps the restart rule proves unchanged (per SKU, the
                             runs up to the first run that changed in the last pass);
                             0: re-evaluate every step each pass.  Same results. */
    int32_t graph_unroll; /* passes per captured HIP graph replay; 0 = automatic,
                             1 = no graph (one host check per pass) */
    const int32_t *init_cache; /* nullable [total], values in [-1, N): alpha^0 in time
                                  order; NULL = lost sale everywhere (Algorithm 1) */
    int32_t validate;     /* nonzero: device range checks of the inputs */
    const int32_t *partition; /* nullable [total], values >= 0: the process of every order
                                 (time order), any assignment, e.g. the uniform random
                                 partitions of Section 4.1; block_len is then ignored.
                                 A process may own several runs of one SKU; each run
                                 starts from the state its process reaches under
                                 Algorithm 1.  PK_ERR_INVALID_ARG for a negative
                                 process. */
    int32_t walk_waves;   /* MLP: waves per workgroup of the run walk, 4 or 8; 0 = the
                             autotuned choice for this problem when block_len is the tuned
                             one, else 4.  Same results either way. */
    int32_t lane_max;     /* greedy, N <= 128, block partitions: in the first pass, runs of
                             at most lane_max orders are walked one per GPU lane (64 runs
                             of similar length per wavefront), longer ones a wavefront per
                             run.  0 = chosen from the workload (the orders per resident
                             lane, up to 510; none below 64); -1 = none; otherwise at most
                             510.  Same results either way. */
} pk_picard_opts;

/* Statistics of one pk_picard_simulate call (all optional). */
typedef struct pk_stats {
    int32_t *passes;         /* HOST nullable [n_traj]: k at which Algorithm 1 returns for
                                each trajectory (its cache stopped changing) */
    int32_t passes_max;      /* passes over the whole batch */
    int32_t block_len;       /* block length used */
    int64_t changed_total;   /* sum over passes of steps whose cached action changed */
    int64_t runs_walked;     /* process runs evaluated (a run: one process's orders of one
                                SKU) */
    int64_t orders_walked;   /* policy evaluations performed over all passes */
    int64_t near_ties;       /* MLP: evaluations (all passes) whose top-two perturbed scores
                                were within 1e-5 relative */
    double walk_ms;          /* summed duration of the policy-evaluation kernel (measured
                                with HIP events on `stream` when timing is requested) */
    int64_t walk_launches;   /* launches of that kernel that did work */
    int64_t walk_bytes;      /* algorithmic HBM bytes of those launches */
    int64_t walk_flops;      /* MLP: algorithmic FLOPs of the rows those launches scored
                                (one row per order and warehouse with stock) */
    int32_t timing;          /* in: nonzero to record walk_ms / walk_bytes */
    double scan_ms;          /* summed duration of the entry-state scan kernel (timing) */
    int64_t scan_launches;   /* launches of that kernel timed */
    int64_t scan_bytes;      /* algorithmic HBM bytes of the scan's launches (u rows read,
                                E rows written, frontier checks) */
    int32_t walk_waves;      /* MLP: waves per workgroup of the run walk used */
} pk_stats;

/* Bytes of scratch that pk_picard_simulate, pk_serial_simulate and pk_policy_grad need
 * for this problem, policy and options (opts nullable = defaults).  Writes *bytes. */
pk_status pk_workspace_size(const pk_problem *problem, const pk_policy *policy,
                            const pk_picard_opts *opts, size_t *bytes);

/* Serial rollout on the GPU (the sequential baseline): one workgroup per trajectory walks
 * t = 1..T in time order, evaluating pi at s_t and applying f.  Same policy code as
 * pk_picard_simulate.
 * actions  [total] out: a_t in [-1, N)
 * shipped  [total] out, nullable: units shipped, min(q_t, x[k_t][a_t]) (0 for a lost sale)
 * final_inv [n_traj][K][N] out, nullable: inventory after the last order. */
pk_status pk_serial_simulate(const pk_problem *problem, const pk_policy *policy, void *ws,
                             size_t ws_bytes, int32_t *actions, int32_t *shipped,
                             int32_t *final_inv, int32_t validate, void *stream);

/* Picard iteration (Algorithm 1) to convergence.  Outputs as pk_serial_simulate; on
 * PK_OK they equal the serial rollout.  On PK_ERR_NOT_CONVERGED, actions hold the cache
 * after max_passes passes (shipped and final_inv are then unspecified) and stats, if
 * given, are filled.  stats: HOST, nullable. */
pk_status pk_picard_simulate(const pk_problem *problem, const pk_policy *policy,
                             const pk_picard_opts *opts, void *ws, size_t ws_bytes,
                             int32_t *actions, int32_t *shipped, int32_t *final_inv,
                             pk_stats *stats, void *stream);

/* Size of the static scratch buffer of pk_picard_simulate_noalloc (64 MiB per device
 * the library runs on, held until the process ends). */
#define PK_NOALLOC_SCRATCH_BYTES (64u << 20)

/* pk_picard_simulate without a workspace and without any allocation, for callers that
 * cannot allocate memory: serving loops that must not call hipMalloc, harnesses that
 * forbid it.  Same problem, policy, options and outputs as pk_picard_simulate; its scratch
 * is a static device buffer of PK_NOALLOC_SCRATCH_BYTES inside the library (one per
 * device, its address resolved on the first call on that device).  The call creates no
 * HIP graph, event or pinned buffer: its passes are enqueued directly on `stream`, and it
 * blocks until the result is final (so it cannot itself be captured into a graph).
 * Differences from pk_picard_simulate:
 *   - block_len 0 takes the library default (1024 greedy, 256 MLP) without autotuning;
 *   - stats->timing must be 0 (PK_ERR_UNSUPPORTED otherwise); walk_ms stays 0;
 *   - PK_ERR_WORKSPACE if the problem needs more than PK_NOALLOC_SCRATCH_BYTES of scratch
 *     (pk_workspace_size reports at least that need; about 1e6 orders at N = 100 fit).
 * Every call on one device shares that device's buffer and overwrites it: calls that
 * overlap in time on one device (other threads, other streams) race and give undefined
 * results; serialise them.  Each call initialises every part of the buffer it reads. */
pk_status pk_picard_simulate_noalloc(const pk_problem *problem, const pk_policy *policy,
                                     const pk_picard_opts *opts, int32_t *actions,
                                     int32_t *shipped, int32_t *final_inv, pk_stats *stats,
                                     void *stream);

/* REINFORCE at fixed actions (MLP policy only).  With the states s_t the actions induce
 * (serially, per trajectory) and pi(.|s) = softmax over warehouses with stock of s_w,
 *   logp[t] = log pi(a_t | s_t)  (0 when at most one warehouse has stock; then a_t must
 *             be the lost sale iff none has),
 *   grad    = d/dparams sum_t advantages[t] * logp[t], same layout as params.
 * Activations are recomputed from the parameters, not stored.
 * actions [total] in (must be feasible at their states, else PK_ERR_INVALID_ARG when
 *         validate is set); advantages [total] in;
 * logp [total] out, nullable; grad [n_params] out, nullable (float32; the sum is
 * accumulated in float64); objective (HOST, nullable) out: sum_t A_t logp[t]. */
pk_status pk_policy_grad(const pk_problem *problem, const pk_policy *policy,
                         const int32_t *actions, const float *advantages, float *logp,
                         float *grad, double *objective, void *ws, size_t ws_bytes,
                         int32_t validate, void *stream);

/* Choose block_len (and, for the MLP policy, the run walk's waves per workgroup) for
 * pk_picard_simulate by timing candidates on this instance (outputs are discarded).
 * Greedy: every candidate length from 64 to 65536, best of three rounds.  MLP: whole
 * simulations, from 2048 up and then down by factors of two while the time falls (a
 * candidate is abandoned once it is slower than the best), then 8 waves per workgroup at
 * the best length.  Results are cached per (policy, N, R, K, total and horizon buckets) in
 * this process, read from the JSON file named by $PICARD_AUTOTUNE_CACHE if set, else from
 * autotune_mi355x.json beside the library (results the autotuner recorded on MI355X),
 * and new results are written to $PICARD_AUTOTUNE_CACHE only.  best_block_len: HOST out. */
pk_status pk_autotune(const pk_problem *problem, const pk_policy *policy, void *ws,
                      size_t ws_bytes, int32_t *best_block_len, void *stream);

/* Diagnostic: noise-free MLP scores s_w of every warehouse w for an order of region
 * `region` in trajectory `traj` at SKU inventory row inv_row ([N], device), written to
 * scores ([N], device, float32).  Same scorer as the simulation kernels.  MLP only. */
pk_status pk_policy_scores(const pk_problem *problem, const pk_policy *policy, int32_t traj,
                           int32_t region, const int32_t *inv_row, float *scores, void *ws,
                           size_t ws_bytes, void *stream);

/* Policy-gradient loop around the rollout (Section 4.2: each iteration rolls out the
 * current policy, forms a policy gradient and takes an Adam step).  The three calls below
 * with pk_picard_simulate (warm-started from the previous iterate's actions through
 * pk_picard_opts.init_cache, the cache choice of Section 5) and pk_policy_grad make one
 * iteration.
 *
 * Bytes of scratch pk_reinforce_advantages needs for this problem.  Writes *bytes. */
pk_status pk_advantages_workspace_size(const pk_problem *problem, size_t *bytes);

/* REINFORCE advantages of a rollout.  Step t earns the chosen warehouse's margin on the
 * units it ships, r_t = (revenue - cost[a_t][region_t]) * shipped_t, and 0 for a lost
 * sale (the FO model of Section 3 earns the chosen node's reward and nothing for an
 * unserved order; `revenue` is the per-unit price that turns a cost into that reward).
 *   advantages[t] = G_t - mean over the trajectory of G,  G_t = sum_{u >= t} r_u,
 * with G, its sum and the rewards exact in int64 and one rounding at the end:
 * float(double(G_t) - double(sum_b G) / T_b).  Synchronous (blocks until done).
 * actions, shipped [total] in (as pk_picard_simulate writes them);
 * advantages [total] out (float32); returns [n_traj] out, nullable: G at each
 * trajectory's first order (its total reward; 0 for an empty trajectory).
 * PK_ERR_INVALID_ARG if an action or region is out of range, shipped < 0, or a reward
 * exceeds the bound that keeps the int64 sums exact: |r_t| <= min(2^31,
 * 2^62 / (T_max (T_max + 1) / 2)), T_max the longest horizon. */
pk_status pk_reinforce_advantages(const pk_problem *problem, const int32_t *actions,
                                  const int32_t *shipped, int32_t revenue, float *advantages,
                                  int64_t *returns, void *ws, size_t ws_bytes, void *stream);

/* One Adam step (Kingma and Ba, Algorithm 1) on n float32 parameters, in float32:
 *   m <- beta1 m + (1 - beta1) grad,  v <- beta2 v + (1 - beta2) grad^2,
 *   params <- params + dir * lr * (m / (1 - beta1^step)) / (sqrt(v / (1 - beta2^step)) + eps)
 * with dir = +1 when `ascend` is nonzero (maximise the objective whose gradient is grad,
 * as for the REINFORCE surrogate) and -1 otherwise.  The hyperparameters are taken in
 * double so that 1 - beta and the bias corrections are formed exactly before their one
 * rounding to float32 (0.999 as a float would make 1 - beta2 wrong by 1.3e-5 relative).  params, m, v [n] in/out (m and v
 * start at zero before step 1; the caller owns them); grad [n] in.  step >= 1 counts the
 * calls.  Asynchronous on `stream`.  PK_ERR_INVALID_ARG for NULL pointers (n > 0),
 * n < 0, step < 1, beta outside [0, 1), lr < 0 or eps <= 0. */
pk_status pk_adam_step(float *params, const float *grad, float *m, float *v, int64_t n,
                       int32_t step, double lr, double beta1, double beta2, double eps,
                       int32_t ascend, void *stream);

/* ---------------------------------------------------------------------------------
 * Node capacity (Section 3: the FO state is (x_t, c_t); an order of SKU i may go to node
 * j only while c_{t,j} > 0 and x_{t,i,j} > 0, and shipping it lowers both by one, so
 * capacity couples the SKUs).  The policy (pk_cap_policy, nullable: NULL is greedy) picks,
 * among the nodes with both stock and capacity, the least of a score, lowest index on ties;
 * a lost sale iff no node has both.  Scores:
 *  - greedy (gamma_num = 0, no bid prices): cost[w][region] (Section 3.1's myopic policy);
 *  - capacity-dependent (the appendix's ablation), gamma = gamma_num / gamma_den with
 *    0 < gamma_num <= 1000, 1 <= gamma_den <= 1000: rank_r(w) + gamma (N-1) p_w,
 *    rank_r(w) the node's position in the region's (cost, index) order and p_w a shadow
 *    price in one of two readings of the appendix's description: gamma_low = 0:
 *    p_w = 1 - c_w / M, M the largest remaining capacity of any node (every node priced);
 *    gamma_low > 0: p_w = max(0, gamma_low - c_w) / gamma_low (only nodes with less than
 *    gamma_low capacity left are priced).  Compared exactly in 64-bit integers;
 *  - bid prices (bid_inv and/or bid_cap non-NULL, gamma_num = 0): cost[w][region] +
 *    bid_inv[sku][w] + bid_cap[w], fixed prices of the unit of stock and of capacity the
 *    order would use (the dual policy of Section 4.2 with its prices held fixed), each
 *    price in [0, 2^24).
 * Unit demand only (every qty must be 1: the paper's transition), one trajectory
 * (n_traj == 1), N <= 128, costs in [0, 2^24).  capacity: DEVICE [N] int32 >= 0, the
 * capacities c_1.  Other arrays as for pk_picard_simulate.  Inputs are range-checked on
 * the device on every call (PK_ERR_INVALID_ARG names the failing check).
 */
typedef struct {
    int32_t gamma_num;        /* 0: no capacity-dependent price */
    int32_t gamma_den;        /* >= 1 */
    int32_t gamma_low;        /* >= 0, see above */
    int32_t reserved;         /* must be 0 */
    const int32_t *bid_inv;   /* DEVICE [K][N] int32, nullable: price of a unit of SKU k's
                                 stock at node w */
    const int32_t *bid_cap;   /* DEVICE [N] int32, nullable: price of a unit of node w's
                                 capacity */
} pk_cap_policy;

/*
 * Bytes of scratch the two calls below need for this problem and block length (0 =
 * the default, 96).  Writes *bytes. */
pk_status pk_capacity_workspace_size(const pk_problem *problem, const int32_t *capacity,
                                     int32_t block_len, size_t *bytes);

/* Serial rollout with capacity (the comparator: one order at a time in time order).
 * actions [T] out; final_inv [K][N] out, nullable; final_cap [N] out, nullable.
 * Synchronous. */
pk_status pk_serial_simulate_capacity(const pk_problem *problem, const int32_t *capacity,
                                      const pk_cap_policy *policy, void *ws,
                                      size_t ws_bytes, int32_t *actions, int32_t *final_inv,
                                      int32_t *final_cap, void *stream);

/* Algorithm 1 with capacity.  The processes are blocks of block_len consecutive orders in
 * time (1..255; 0 = 96): process m owns orders [m B, (m+1) B).  init_cache [T] DEVICE,
 * nullable (NULL: lost sale everywhere) is alpha^0.  max_passes 0 means T + 1
 * (Proposition 2.1 bounds the passes by T + 1).  On return actions [T] holds the fixed
 * point, which equals pk_serial_simulate_capacity's actions; final_inv [K][N] and
 * final_cap [N] (both nullable) the state after the last order.  passes: HOST out, the
 * pass whose cache repeated the previous one (k* + 1, k* the first pass whose cache is the
 * serial trajectory).  changed: HOST [max_passes] out, nullable: orders whose action
 * changed in each pass.  caches: DEVICE [max_passes][T] out, nullable: alpha^k after pass
 * k.  Synchronous (the pass count is data-dependent).  PK_ERR_NOT_CONVERGED if
 * max_passes passes end without a repeat (actions then holds the last cache and the
 * final state is not written). */
pk_status pk_picard_simulate_capacity(const pk_problem *problem, const int32_t *capacity,
                                      const pk_cap_policy *policy, int32_t block_len, int32_t max_passes,
                                      const int32_t *init_cache, void *ws, size_t ws_bytes,
                                      int32_t *actions, int32_t *final_inv, int32_t *final_cap,
                                      int32_t *passes, int64_t *changed, int32_t *caches,
                                      void *stream);

/* ---------------------------------------------------------------------------------
 * One Warehouse Multi-Retailer inventory control (the appendix's extension "Inventory
 * Control with Replenishment"): one central warehouse and N retailers.  Order t is a
 * demand of d_t >= 0 units at retailer n_t.  The retailer, at stock x before the demand,
 * keeps p = (x - d_t)^+ and orders q = min(S_n, c_n) - p if p <= s_n (and that is
 * positive), else 0; the central warehouse, at stock x_0, resets (orders up to S0) iff
 * x_0 - q <= s0.  The retailer receives min(q, x_0); x_0 becomes S0 after a reset, else
 * (x_0 - q)^+.  The action of order t is (q_t, reset_t).  Integer arithmetic throughout. */
typedef struct pk_owmr_problem {
    int32_t n_retailers;      /* N >= 1 */
    int32_t reserved;         /* 0 */
    int64_t n_orders;         /* T >= 0, < 2^31 */
    const int32_t *retailer;  /* [T] in [0, N) */
    const int32_t *demand;    /* [T] >= 0 */
    const int32_t *s_ret;     /* [N] reorder points s_n */
    const int32_t *S_ret;     /* [N] order-up-to levels S_n >= 0 */
    const int32_t *cap;       /* [N] capacities c_n >= 0, with T c_n < 2^40 */
    const int32_t *x_init;    /* [N] retailer stock at t = 0, in [0, c_n] */
    int64_t s0, S0, x0_init;  /* central (s, S) rule and its stock at t = 0 (S0, x0_init >= 0) */
} pk_owmr_problem;

/* Bytes of scratch the two OWMR calls need.  Writes *bytes. */
pk_status pk_owmr_workspace_size(const pk_owmr_problem *problem, size_t *bytes);

/* The serial rollout (one order at a time, on the GPU).  q, reset [T] out (int32);
 * final_x [N] out, nullable (retailer stock after the last order); final_x0, resets:
 * HOST out, nullable (central stock after the last order; R, the number of resets).
 * PK_ERR_INVALID_ARG for out-of-range inputs (checked on the device).  Synchronous. */
pk_status pk_owmr_serial_simulate(const pk_owmr_problem *problem, void *ws, size_t ws_bytes,
                                  int32_t *q, int32_t *reset, int32_t *final_x,
                                  int64_t *final_x0, int64_t *resets, void *stream);

/* Algorithm 1 with one process per retailer (the appendix's allocation of the orders of
 * retailer n to process n).  init_q, init_reset: DEVICE [T] nullable (NULL: no order and
 * no reset everywhere) is alpha^0.  max_passes 0 means T + 1 (Proposition 2.1).  Outputs
 * as pk_owmr_serial_simulate; on PK_OK they equal the serial rollout.  passes: HOST out
 * (k* + 1).  changed: HOST [max_passes] out, nullable: orders whose action changed in each
 * pass.  caches: DEVICE [max_passes][T] int64 out, nullable: alpha^k after pass k packed as
 * reset * 2^40 + q.  PK_ERR_NOT_CONVERGED when max_passes end without a repeat (q and
 * reset then hold the last cache).  Synchronous. */
pk_status pk_owmr_picard_simulate(const pk_owmr_problem *problem, int32_t max_passes,
                                  const int32_t *init_q, const int32_t *init_reset, void *ws,
                                  size_t ws_bytes, int32_t *q, int32_t *reset, int32_t *final_x,
                                  int64_t *final_x0, int32_t *passes, int64_t *changed,
                                  int64_t *caches, void *stream);

/* Message for the last non-OK status on this thread ("" if none). */
const char *pk_last_error(void);

/* Library version string. */
const char *pk_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PICARD_H */

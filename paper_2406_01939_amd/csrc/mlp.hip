// Learned softmax policy kernels: the MLP scorer on MFMA, the Picard run walk, the serial
// sweep and a diagnostic scorer.
//
// Policy (learned fulfillment policy, trained by policy gradient in Section 4.2): per
// (order, warehouse) row the features [cost[w][r], log1p(x[w]), E[r][0..15]] go through
// h1 = relu(W1 f + b1), h2 = relu(W2 h1 + b2), s = w3 . h + b3 (h = h2, or h1 with one
// hidden layer); the action is argmax over warehouses with stock of s_w + G(t, traj, w)
// (lowest index on exact ties), G a Gumbel variate; this samples softmax(s) over the
// warehouses with stock.  The noise is part of the order's disturbance (Section 2).
//
// Scorer: 16 rows (warehouses of one order) per wave step, in transposed form so that a
// layer's MFMA output registers are directly the next layer's MFMA input:
//   H1^T[64 x 16] = W1[64 x 20] F^T[20 x 16]    (features padded 18 -> 20)
//   H2^T[64 x 16] = W2[64 x 64] H1^T[64 x 16]
// with v_mfma_f32_16x16x4f32 (A: lane l holds A[l%16][l/16]; B: lane l holds
// B[l/16][l%16]; D: lane l, register v holds D[4(l/16)+v][l%16]).  Lane l keeps hidden
// units 16t + 4(l/16) + v of row l%16, so layer 2 sums its k dimension in the order
// h = 16(s/4) + 4(l/16) + s%4 over its 16 steps s; W2's A operand is loaded in that
// order.  The accumulation order of every row's dot products is fixed, so a row's score
// does not depend on which other rows share its tile (the walk and the serial sweep
// produce bit-identical scores).
#include "mlp_device.h"

namespace pk {

namespace {

using namespace mlpdev;

// The region terms of layer 1, W1[:,2:] E[r] + b1, follow the cost rows in the same
// buffer: [R][64] floats after costT[n_traj][R][N].
__device__ __forceinline__ const float *region_table(const float *costT, const Prob &P)
{
    return costT + (int64_t)P.n_traj * P.R * P.N;
}

// Per-order data of both learned kernels comes from LDS: the orders of a run (or a
// trajectory) are staged 64 at a time, the next 64 loaded into registers meanwhile, and
// each order's cost row and region embedding sit in a double buffer that is filled from
// global memory while the previous order is scored.  CHUNK orders per stage.
constexpr int CHUNK = 64;
// Loads the cost row of region r (N values, trajectory b) into registers (CPT values per
// thread of a THREADS-thread workgroup).
template <int THREADS, int CPT = PK_MAX_WAREHOUSES / THREADS>
__device__ __forceinline__ void load_row(const float *costT, int b, int R, int N, int r,
                                         float cn[CPT])
{
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        const int w = k * THREADS + (int)threadIdx.x;
        cn[k] = w < N ? costT[((int64_t)b * R + r) * N + w] : 0.f;
    }
}
template <int THREADS, int CPT = PK_MAX_WAREHOUSES / THREADS>
__device__ __forceinline__ void store_row(float *cbuf, int N, const float cn[CPT])
{
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        const int w = k * THREADS + (int)threadIdx.x;
        if (w < N) cbuf[w] = cn[k];
    }
}

// One workgroup walks one run (a process's orders of one SKU) from its entry state,
// order by order: all waves score the order's warehouses with stock (kept as a list that
// loses a warehouse when it empties), wave 0 takes the argmax and applies f.  Same run bookkeeping as the greedy walk (entry state from the segmented
// scan, u of split runs, final inventory of a SKU's last run, restart frontier).  Under a
// given partition the workgroup goes on to its process's later runs of the SKU (its
// chain), entering each at max(0, x0 - E_j - D), D the process's own fresh-minus-cached
// consumption on its earlier runs, kept in LDS.
// WPB waves per workgroup (4 or 8): the tiles of an order are shared by more waves with 8
// (shorter orders, for wide N), at half the resident workgroups per CU (four waves per SIMD
// either way).
template <int WPB>
__global__ __launch_bounds__(WPB * 64, 16 / WPB) void k_walk_mlp(Prob P, Plan L, const float *params, int layers,
                                                  const float *costT, int32_t *final_inv,
                                                  int has_init)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = P.N, R = P.R;
    float *W2s = (float *)smem;
    float *Vs = (float *)(smem + w2_lds_bytes());
    int32_t *x = (int32_t *)(smem + w2_lds_bytes() + vec_lds_bytes());
    int32_t *cons = x + N;
    float *zbuf = (float *)(cons + N);
    int32_t *sl = (int32_t *)(zbuf + N); // warehouses with stock
    int32_t *pos = sl + N;               // index of each in sl
    int32_t *flag = pos + N;             // [0] changed, [1] near ties, [2] stock list length
    int32_t *dcor = flag + 4;            // given partitions: the process's own correction
    float *lxs = (float *)(dcor + N);    // log1p of each warehouse's stock (feature cache)
    float *cbs = lxs + N;                // [2][N] cost rows of this order's and the next's region
    float *prs = (float *)(((uintptr_t)(cbs + 2 * N) + 15) & ~(uintptr_t)15); // [2][64] their
                                         // region terms of layer 1
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    Ctl *ctl = L.ctl;
    if (ctl->done) return;
    stage_w2(W2s, params, R, layers); // both read after the first barrier of a run
    stage_vectors(Vs, params, R, layers);
    ScoreLane m;
    load_score_lane(m, params, R, layers, W2s, Vs);
    const float *rtab = region_table(costT, P); // [R][64] region terms of layer 1
    const int pass = ctl->pass;
    const int32_t *fprev = L.fr[(pass - 1) & 1];
    int32_t *fcur = L.fr[pass & 1];
    const bool first = pass == 1;
    const bool all = first || L.no_frontier;
    const int n_items = all ? ctl->n_sr : ctl->n_split;
    const bool need_E = !first || has_init;
    int lcp_b = -1; // last trajectory this wave marked as changed in this pass
    unsigned long long n_orders = 0, n_runs = 0, n_changed = 0, n_bytes = 0, n_ties = 0;
    unsigned long long n_rows = 0; // scored (order, warehouse with stock) rows
    // one loop over the runs this workgroup walks: the next item's run, or under a given
    // partition the next run of the current chain
    int item = blockIdx.x, s_next = -1;
    for (;;) {
        int s = s_next;
        s_next = -1;
        if (s < 0) {
            if (item >= n_items) break;
            s = all ? item : L.split_list[item];
            item += gridDim.x;
            const int g = L.sr_seg[s];
            const int32_t f = all ? FR_ALL : fprev[g];
            if (!all && (f == FR_NONE || s - L.seg_sr0[g] <= f)) continue;
            // a given partition's chain is walked from its first run past the frontier
            // (the process's earlier runs keep their actions and add nothing to D)
            if (L.worker && L.ch_prevj[s] > f) continue;
            if (L.worker)
                for (int w = threadIdx.x; w < N; w += blockDim.x) dcor[w] = 0;
        }
        const int g = L.sr_seg[s];
        const int s0 = L.seg_sr0[g];
        const int j = s - s0;
        const int nsr = L.seg_sr0[g + 1] - s0;
        const int lo = L.sr_lo[s], hi = L.sr_lo[s + 1];
        const int key = L.seg_key[g];
        const int b = key / P.K;
        const int32_t *x0row = P.x0 + (int64_t)key * N;
        const int uidx = L.sr_uidx[s];
        const int32_t *Erow = (need_E && j > 0) ? L.E + (int64_t)uidx * N : nullptr;
        __syncthreads(); // dcor is final (set above, or by the chain's previous run)
        for (int w = threadIdx.x; w < N; w += blockDim.x) {
            const int32_t v = x0row[w] - (Erow ? Erow[w] : 0) - (L.worker ? dcor[w] : 0);
            x[w] = v > 0 ? v : 0;
            lxs[w] = log1p_stock(v > 0 ? v : 0);
            cons[w] = 0;
        }
        // the first order's region rows into buffer 0; the next order's region and time
        const int rn = L.s_region[lo];
        uint32_t tn = (uint32_t)L.s_t[lo];
        for (int w = threadIdx.x; w < N; w += blockDim.x) cbs[w] = costT[((int64_t)b * R + rn) * N + w];
        if (threadIdx.x < 64) prs[threadIdx.x] = rtab[(int64_t)rn * 64 + threadIdx.x];
        int r1 = lo + 1 < hi ? L.s_region[lo + 1] : 0;
        uint32_t t1 = lo + 1 < hi ? (uint32_t)L.s_t[lo + 1] : 0u;
        __syncthreads();
        build_stock_list(x, N, sl, pos, &flag[2]);
        __syncthreads();
        int nf = flag[2];       // wave 0 keeps the list length; the others reread it
        int run_chg = 0, run_ties = 0; // wave 0, lane 0
        for (int p = lo; p < hi; ++p) {
            const int cur = (p - lo) & 1;
            const uint32_t t = tn;
            const bool hn = p + 1 < hi;
            // the region and time of the order after the next one
            const int r2 = p + 2 < hi ? L.s_region[p + 2] : 0;
            const uint32_t t2 = p + 2 < hi ? (uint32_t)L.s_t[p + 2] : 0u;
            // wave 0's lane 0 needs the order's quantity and cached action after the argmax
            int q = 0, old = 0;
            if (threadIdx.x == 0) {
                q = L.s_qty[p];
                old = L.s_alpha[p];
            }
            if (wave != 0) nf = flag[2];
            float pr[16];
            load_region_term(pr, prs + cur * 64, 0);
            score_rows(m, pr, cbs + cur * N, x, lxs, sl, nf, P.seed, (uint32_t)b, t, zbuf);
            __syncthreads();
            if (wave == 0) {
                float z1, z2;
                const int a = argmax_zl(zbuf, sl, nf, z1, z2);
                int emp = 0;
                if (lane == 0) {
                    int sh = 0;
                    if (a >= 0) { // the four reads are independent: one round trip
                        const int xa = x[a], ca = cons[a], ia = pos[a], last = sl[nf - 1];
                        sh = q < xa ? q : xa;
                        x[a] = xa - sh;
                        lxs[a] = log1p_stock(xa - sh);
                        cons[a] = ca + q;
                        if (xa == sh) { // emptied: the list's last entry takes its place
                            sl[ia] = last;
                            pos[last] = ia;
                            flag[2] = nf - 1;
                            emp = 1;
                        }
                    }
                    n_rows += nf;
                    run_chg += old != a;
                    run_ties += near_tie(z1, z2);
                    L.s_alpha[p] = a;
                    L.s_ship[p] = sh;
                    if (L.worker) { // own correction: fresh minus cached
                        if (a >= 0) dcor[a] += q;
                        if (old >= 0) dcor[old] -= q;
                    }
                }
                nf -= __builtin_amdgcn_readlane(emp, 0);
            }
            if (wave != 0 && hn) {
                // the next order's region rows into the other buffer (last read by the
                // previous order's tiles) while wave 0 takes this order's argmax: all
                // loads of a round issued before their stores
                constexpr int NT = (WPB - 1) * WAVE;
                const int tid = (int)threadIdx.x - WAVE;
                const float *src = costT + ((int64_t)b * R + r1) * N;
                float *dst = cbs + (cur ^ 1) * N;
                for (int base = 0; base < N; base += 4 * NT) {
                    float cv[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int w = base + k * NT + tid;
                        cv[k] = w < N ? src[w] : 0.f;
                    }
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int w = base + k * NT + tid;
                        if (w < N) dst[w] = cv[k];
                    }
                }
                if (tid < 64) prs[(cur ^ 1) * 64 + tid] = rtab[(int64_t)r1 * 64 + tid];
            }
            tn = t1;
            r1 = r2;
            t1 = t2;
            __syncthreads();
        }
        if (threadIdx.x == 0) { flag[0] = run_chg; flag[1] = run_ties; }
        __syncthreads();
        int wr = 0;
        if (uidx >= 0) {
            for (int w = threadIdx.x; w < N; w += blockDim.x) L.u[(int64_t)uidx * N + w] = cons[w];
            ++wr;
        }
        if (final_inv && j == nsr - 1) {
            for (int w = threadIdx.x; w < N; w += blockDim.x) final_inv[(int64_t)key * N + w] = x[w];
            ++wr;
        }
        if (threadIdx.x == 0) {
            const int nchg = flag[0];
            if (nchg) {
                atomicMin(&fcur[g], j);
                if (b != lcp_b) { // once per trajectory in a row; read first (one hot word)
                    if (L.traj_lcp[b] < pass) atomicMax(&L.traj_lcp[b], pass);
                    lcp_b = b;
                }
            }
            n_changed += nchg;
            n_ties += flag[1];
            n_orders += hi - lo;
            n_runs += 1;
            n_bytes += 24ull * (hi - lo) + 4ull * N * (1 + (Erow ? 1 : 0) + wr);
        }
        __syncthreads();
        if (L.worker) {
            const int nx = L.ch_next[s];
            if (nx > s && nx < ctl->n_sr) s_next = nx;
            else if (nx >= 0 && threadIdx.x == 0) // links always point forward: never loop
                atomicOr(&ctl->error, ERR_NO_PROGRESS);
        }
    }
    if (threadIdx.x == 0 && n_runs) {
        unsigned long long *st = ctl->stat[blockIdx.x % STAT_SLOTS];
        atomicAdd(&st[ST_ORDERS], n_orders);
        atomicAdd(&st[ST_RUNS], n_runs);
        atomicAdd(&st[ST_CHANGED], n_changed);
        atomicAdd(&st[ST_BYTES], n_bytes);
        atomicAdd(&st[ST_NEAR_TIES], n_ties);
        atomicAdd(&st[ST_FLOPS], n_rows * row_flops(layers));
    }
    walk_finish(ctl, lcp_b >= 0);
}

// Serial sweep: one workgroup per trajectory walks its orders in time order with the
// trajectory's stock in `state` ([K][N], initialised to x0); per order the SKU's stock
// row is in LDS (requested during the previous order, or kept from it when both orders
// have the same SKU), its warehouses with stock are listed and scored by the same scorer,
// and the chosen warehouse's stock is written back.
template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_serial_mlp(Prob P, const float *params, int layers,
                                                       const float *costT, int32_t *state,
                                                       int32_t *actions, int32_t *shipped)
{
    constexpr int CPT = PK_MAX_WAREHOUSES / THREADS; // cost and stock values per thread
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = P.N, R = P.R;
    float *W2s = (float *)smem;
    float *Vs = (float *)(smem + w2_lds_bytes());
    int4 *ordq = (int4 *)(smem + w2_lds_bytes() + vec_lds_bytes()); // [2][CHUNK] (k, r, q, -)
    float *cbuf = (float *)(ordq + 2 * CHUNK); // [2][N]
    int32_t *x = (int32_t *)(cbuf + 2 * N);
    float *zbuf = (float *)(x + N);
    int32_t *sl = (int32_t *)(zbuf + N);
    int32_t *pos = sl + N;
    int32_t *nfp = pos + N;
    const int b = blockIdx.x;
    if (b >= P.n_traj) return;
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int tid = threadIdx.x;
    stage_w2(W2s, params, R, layers); // both read after the first barrier
    stage_vectors(Vs, params, R, layers);
    ScoreLane m;
    load_score_lane(m, params, R, layers, W2s, Vs);
    const float *rtab = region_table(costT, P);
    const int64_t t0 = P.traj_off[b], t1 = P.traj_off[b + 1];
    int32_t *xs = state + (int64_t)b * P.K * N;
    auto order_at = [&](int64_t t) -> int4 {
        int k = P.sku[t], r = P.region[t], q = P.qty[t];
        k = k < 0 ? 0 : (k >= P.K ? P.K - 1 : k); // out-of-range input never indexes memory
        r = r < 0 ? 0 : (r >= P.R ? P.R - 1 : r);
        q = q < 1 ? 1 : q;
        return make_int4(k, r, q, 0);
    };
    if (t0 >= t1) return;
    if (tid < CHUNK && t0 + tid < t1) ordq[tid] = order_at(t0 + tid);
    int4 nq = make_int4(0, 0, 0, 0);
    if (tid < CHUNK && t0 + CHUNK + tid < t1) nq = order_at(t0 + CHUNK + tid);
    __syncthreads();
    float cn[CPT];
    load_row<THREADS>(costT, b, R, N, ordq[0].y, cn);
    store_row<THREADS>(cbuf, N, cn);
    for (int w = tid; w < N; w += blockDim.x) x[w] = xs[(int64_t)ordq[0].x * N + w];
    __syncthreads();
    for (int64_t tt = t0; tt < t1; ++tt) {
        const int64_t i = tt - t0;
        const int slot = (int)((i / CHUNK) & 1), buf = (int)(i & 1);
        if (i % CHUNK == 0 && i > 0) { // a new chunk: into the ring, the next one requested
            if (tid < CHUNK) ordq[slot * CHUNK + tid] = nq;
            if (tid < CHUNK && tt + CHUNK + tid < t1) nq = order_at(tt + CHUNK + tid);
            __syncthreads();
            // this order's rows were not prefetched: its cost row, and its stock row as the
            // previous order left it (written back before the last barrier)
            const int4 o0 = ordq[slot * CHUNK];
            load_row<THREADS>(costT, b, R, N, o0.y, cn);
            store_row<THREADS>(cbuf + buf * N, N, cn);
            for (int w = tid; w < N; w += blockDim.x) x[w] = xs[(int64_t)o0.x * N + w];
            __syncthreads();
        }
        const int4 od = ordq[slot * CHUNK + (int)(i % CHUNK)];
        const int k = od.x, q = od.z;
        int32_t *xk = xs + (int64_t)k * N;
        // the next order (same chunk): its row and, for another SKU, its stock row
        const bool pf = i % CHUNK != CHUNK - 1 && tt + 1 < t1;
        int kn = k;
        int32_t xn[CPT];
        if (pf) {
            const int4 on = ordq[slot * CHUNK + (int)(i % CHUNK) + 1];
            kn = on.x;
            load_row<THREADS>(costT, b, R, N, on.y, cn);
            if (kn != k) {
#pragma unroll
                for (int c = 0; c < CPT; ++c) {
                    const int w = c * THREADS + tid;
                    xn[c] = w < N ? xs[(int64_t)kn * N + w] : 0;
                }
            }
        }
        build_stock_list(x, N, sl, pos, nfp);
        __syncthreads();
        const int nf = *nfp;
        float pr[16];
        load_region_term(pr, rtab, od.y);
        score_rows(m, pr, cbuf + buf * N, x, nullptr, sl, nf, P.seed, (uint32_t)b, (uint32_t)(tt - t0),
                   zbuf);
        __syncthreads();
        if (wave == 0) {
            float z1, z2;
            const int a = argmax_zl(zbuf, sl, nf, z1, z2);
            if (lane == 0) {
                int sh = 0;
                if (a >= 0) {
                    sh = q < x[a] ? q : x[a];
                    x[a] -= sh;
                    xk[a] = x[a];
                }
                actions[tt] = a;
                if (shipped) shipped[tt] = sh;
            }
        }
        __syncthreads();
        // the next order's rows into LDS: its stock row is kept when it is the same SKU
        // (updated above); when the next order opens a chunk both are read there
        if (pf) {
            store_row<THREADS>(cbuf + (buf ^ 1) * N, N, cn);
            if (kn != k) {
#pragma unroll
                for (int c = 0; c < CPT; ++c) {
                    const int w = c * THREADS + tid;
                    if (w < N) x[w] = xn[c];
                }
            }
        }
        __threadfence_block();
        __syncthreads();
    }
}

// Diagnostic: raw scores s_w (no noise) of every warehouse for region r of trajectory b at
// inventory row xrow; one workgroup.
__global__ __launch_bounds__(256) void k_scores(Prob P, const float *params, int layers,
                                                const float *costT, int b, int r,
                                                const int32_t *xrow, float *out)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = P.N;
    float *W2s = (float *)smem;
    float *Vs = (float *)(smem + w2_lds_bytes());
    int32_t *x = (int32_t *)(smem + w2_lds_bytes() + vec_lds_bytes());
    float *zbuf = (float *)(x + N);
    float *sbuf = zbuf + N;
    stage_w2(W2s, params, P.R, layers); // both read after the barrier below
    stage_vectors(Vs, params, P.R, layers);
    ScoreLane m;
    load_score_lane(m, params, P.R, layers, W2s, Vs);
    for (int w = threadIdx.x; w < N; w += blockDim.x) x[w] = xrow[w];
    __syncthreads();
    float pr[16];
    load_region_term(pr, region_table(costT, P), r);
    score_all(m, pr, costT + ((int64_t)b * P.R + r) * N, x, N, sbuf);
    (void)zbuf;
    __syncthreads();
    for (int w = threadIdx.x; w < N; w += blockDim.x) out[w] = sbuf[w];
}

// costT[b][r][w] = (float)cost[b][w][r]: each order's cost row contiguous.
__global__ void k_cost_t(Prob P, float *costT)
{
    const int64_t n = (int64_t)P.n_traj * P.R * P.N;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int w = (int)(i % P.N);
        const int64_t br = i / P.N;
        const int r = (int)(br % P.R);
        const int64_t b = br / P.R;
        costT[i] = (float)P.cost[(b * P.N + w) * P.R + r];
    }
}

// Region terms of layer 1: table[r][u] = b1[u] + sum_i W1[u][2 + i] E[r][i], summed in
// FP32 in the order i = 0..15 (one thread per (r, u)).
__global__ void k_region_l1(const float *params, int R, float *table)
{
    const int64_t n = (int64_t)R * 64;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const float *W1 = params + (int64_t)R * 16;
    const float *b1 = W1 + 64 * 18;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int u = (int)(i & 63);
        const int64_t r = i >> 6;
        float acc = b1[u];
#pragma unroll
        for (int k = 0; k < 16; ++k) acc = fmaf(W1[u * 18 + 2 + k], params[r * 16 + k], acc);
        table[i] = acc;
    }
}

} // namespace

size_t costT_bytes(int N, int R, int n_traj)
{
    return ((size_t)n_traj * R * N + (size_t)R * 64) * sizeof(float);
}

hipError_t setup_costT(const Prob &P, const float *params, float *costT, hipStream_t st)
{
    const int64_t n = (int64_t)P.n_traj * P.R * P.N;
    int64_t g = (n + 255) / 256;
    g = g < 1 ? 1 : (g > 8192 ? 8192 : g);
    hipLaunchKernelGGL(k_cost_t, dim3((unsigned)g), dim3(256), 0, st, P, costT);
    const int64_t nr = (int64_t)P.R * 64;
    int64_t gr = (nr + 255) / 256;
    gr = gr < 1 ? 1 : (gr > 4096 ? 4096 : gr);
    hipLaunchKernelGGL(k_region_l1, dim3((unsigned)gr), dim3(256), 0, st, params, P.R,
                       costT + n);
    return hipGetLastError();
}

size_t walk_mlp_lds(int N) { return w2_lds_bytes() + vec_lds_bytes() + (size_t)N * 36 + 64 + 16 + 512; }

hipError_t launch_walk_mlp(const Prob &P, const Plan &L, const float *params, int layers,
                           const float *costT, int32_t *final_inv, bool has_init, int n_cus,
                           int waves, hipStream_t st)
{
    // persistent: as many workgroups as stay resident (four waves per SIMD)
    if (waves == 8)
        hipLaunchKernelGGL(k_walk_mlp<8>, dim3(n_cus * 2), dim3(512), walk_mlp_lds(P.N), st, P, L,
                           params, layers, costT, final_inv, has_init ? 1 : 0);
    else
        hipLaunchKernelGGL(k_walk_mlp<4>, dim3(n_cus * 4), dim3(256), walk_mlp_lds(P.N), st, P, L,
                           params, layers, costT, final_inv, has_init ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_serial_mlp(const Prob &P, const float *params, int layers, const float *costT,
                             int32_t *state, int32_t *actions, int32_t *shipped, hipStream_t st)
{
    // a trajectory's orders go one at a time, so its workgroup should score each order's
    // tiles with as many waves as the tiles keep busy: 16 waves for wide orders, else 4
    const size_t lds = w2_lds_bytes() + vec_lds_bytes() + (size_t)2 * CHUNK * 16 +
                       (size_t)P.N * 24 + 64;
    if (P.N > 256)
        hipLaunchKernelGGL(k_serial_mlp<1024>, dim3(P.n_traj), dim3(1024), lds, st, P, params,
                           layers, costT, state, actions, shipped);
    else
        hipLaunchKernelGGL(k_serial_mlp<256>, dim3(P.n_traj), dim3(256), lds, st, P, params,
                           layers, costT, state, actions, shipped);
    return hipGetLastError();
}

hipError_t launch_scores(const Prob &P, const float *params, int layers, const float *costT,
                         int b, int r, const int32_t *xrow, float *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_scores, dim3(1), dim3(256),
                       w2_lds_bytes() + vec_lds_bytes() + (size_t)P.N * 12 + 64, st, P,
                       params, layers,
                       costT, b, r, xrow, out);
    return hipGetLastError();
}

} // namespace pk

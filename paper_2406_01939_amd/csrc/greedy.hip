// Greedy policy kernels: the Picard run walk and the serial sweep.
//
// Greedy (Section 3.1, inventory as the constraint): among warehouses with stock, the
// least cost[w][region], lowest index on ties; lost sale iff none has stock.  With
// rank[b][r] listing warehouses by (cost, index), the choice is the first warehouse of
// rank[b][r] with stock.
#include "pk_internal.h"

namespace pk {

namespace {

constexpr int UNKNOWN = -2;

// One wave walks one run (a process's orders of one SKU) from its entry state, exactly
// as Algorithm 1's process does, 64 orders at a time:
//  * every lane takes the choice its order would get at the chunk's starting state (a
//    per-region "best warehouse" memo, refreshed when its warehouse empties);
//  * the chunk's demand per chosen warehouse is summed in LDS; a warehouse whose demand
//    exceeds its stock empties inside the chunk, and the first order that finds it
//    empty (exclusive prefix of demand >= stock) is the first order whose choice is no
//    longer valid;
//  * all orders before it are exact (stock only falls, so a choice changes only when
//    the chosen warehouse empties); they are committed and the walk resumes there.
// Per wave LDS: x[N] stock, tot[N] chunk demand, cons[N] run consumption (unclamped, for
// u), bw[R] / bj[R] memoised best warehouse and its rank position per region.
__global__ __launch_bounds__(256) void k_walk_greedy(Prob P, Plan L, int32_t *final_inv,
                                                     int has_init)
{
    extern __shared__ int32_t lds[];
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int N = P.N, R = P.R;
    int32_t *x = lds + wave * (3 * N + 2 * R);
    int32_t *tot = x + N;
    int32_t *cons = tot + N;
    int32_t *bw = cons + N;
    int32_t *bj = bw + R;
    Ctl *ctl = L.ctl;
    if (ctl->done) return;
    const int pass = ctl->pass;
    const int32_t *fprev = L.fr[(pass - 1) & 1];
    int32_t *fcur = L.fr[pass & 1];
    const bool first = pass == 1;
    const int n_items = first ? ctl->n_sr : ctl->n_split;
    const bool need_E = !first || has_init;
    unsigned long long n_orders = 0, n_runs = 0, n_changed = 0, n_bytes = 0;

    for (;;) {
        int item = 0;
        if (lane == 0) item = atomicAdd(&ctl->work, 1);
        item = __shfl(item, 0, WAVE);
        if (item >= n_items) break;
        const int s = first ? item : L.split_list[item];
        const int g = L.sr_seg[s];
        const int s0 = L.seg_sr0[g];
        const int j = s - s0;
        if (!first) {
            const int32_t f = fprev[g];
            if (f == FR_NONE || j <= f) continue;
        }
        const int nsr = L.seg_sr0[g + 1] - s0;
        const int lo = L.sr_lo[s], hi = L.sr_lo[s + 1];
        const int key = L.seg_key[g];
        const int b = key / P.K;
        const int32_t *x0row = P.x0 + (int64_t)key * N;
        const int uidx = L.sr_uidx[s];
        const int32_t *Erow = (need_E && j > 0) ? L.E + (int64_t)uidx * N : nullptr;
        for (int w = lane; w < N; w += WAVE) {
            const int32_t v = x0row[w] - (Erow ? Erow[w] : 0);
            x[w] = v > 0 ? v : 0;
            tot[w] = 0;
            cons[w] = 0;
        }
        for (int r = lane; r < R; r += WAVE) bw[r] = UNKNOWN;
        wave_sync();
        const int16_t *rank_b = L.rank + (int64_t)b * R * N;
        bool changed = false;
        int p = lo;
        while (p < hi) {
            const int n = hi - p < WAVE ? hi - p : WAVE;
            const bool act = lane < n;
            int r = 0, q = 0, old = 0, a = LOST;
            if (act) {
                r = L.s_region[p + lane];
                q = L.s_qty[p + lane];
                old = L.s_alpha[p + lane];
                int w = bw[r];
                if (w == UNKNOWN || (w >= 0 && x[w] <= 0)) {
                    int jj = w == UNKNOWN ? 0 : bj[r] + 1;
                    const int16_t *rk = rank_b + (int64_t)r * N;
                    w = LOST;
                    for (; jj < N; ++jj) {
                        const int c = rk[jj];
                        if (x[c] > 0) { w = c; break; }
                    }
                    bw[r] = w;
                    bj[r] = jj;
                }
                a = w;
            }
            wave_sync();
            if (act && a >= 0) atomicAdd(&tot[a], q);
            wave_sync();
            const bool flag = act && a >= 0 && tot[a] > x[a];
            uint64_t todo = __ballot(flag);
            int cut = n;
            int ship = q;
            while (todo) {
                const int l0 = __ffsll((long long)todo) - 1;
                const int w0 = __shfl(a, l0, WAVE);
                const bool mine = act && a == w0;
                const uint64_t eq = __ballot(mine);
                const int qq = mine ? q : 0;
                const int excl = wave_incl_sum(qq) - qq;
                const int xw = x[w0];
                const bool invalid = mine && excl >= xw;
                if (mine && !invalid) ship = q < xw - excl ? q : xw - excl;
                const uint64_t inv = __ballot(invalid);
                if (inv) {
                    const int c = __ffsll((long long)inv) - 1;
                    cut = c < cut ? c : cut;
                }
                todo &= ~eq;
            }
            const bool commit = act && lane < cut;
            if (commit) {
                L.s_alpha[p + lane] = a;
                L.s_ship[p + lane] = a >= 0 ? ship : 0;
                changed |= a != old;
            }
            n_changed += __popcll(__ballot(commit && a != old));
            wave_sync();
            if (commit && a >= 0) {
                atomicSub(&x[a], ship);
                atomicAdd(&cons[a], q);
            }
            if (act && a >= 0) tot[a] = 0;
            wave_sync();
            p += cut;
        }
        wave_sync();
        int wr = 0;
        if (uidx >= 0) {
            for (int w = lane; w < N; w += WAVE) L.u[(int64_t)uidx * N + w] = cons[w];
            ++wr;
        }
        if (final_inv && j == nsr - 1) {
            for (int w = lane; w < N; w += WAVE) final_inv[(int64_t)key * N + w] = x[w];
            ++wr;
        }
        const bool any = __ballot(changed) != 0;
        if (lane == 0) {
            if (any) {
                atomicMin(&fcur[g], j);
                atomicMax(&L.traj_lcp[b], pass);
                ctl->any_changed = 1;
            }
            n_orders += hi - lo;
            n_runs += 1;
            n_bytes += 20ull * (hi - lo) + 4ull * N * (1 + (Erow ? 1 : 0) + wr);
        }
        wave_sync();
    }
    if (lane == 0 && n_runs) {
        atomicAdd(&ctl->orders_walked, n_orders);
        atomicAdd(&ctl->runs_walked, n_runs);
        atomicAdd(&ctl->changed_this_pass, n_changed);
        atomicAdd(&ctl->bytes_walked, n_bytes);
    }
}

// Serial sweep: one wave per trajectory walks its orders in time order.  The stock of
// the trajectory lives in `state` ([K][N], initialised to x0); per order the wave reads
// the region's rank row 64 positions at a time and takes the first warehouse with stock
// (ballot), and lane 0 applies f.  The store is fenced before the next order's loads.
__global__ __launch_bounds__(64) void k_serial_greedy(Prob P, const int16_t *rank,
                                                      int32_t *state, int32_t *actions,
                                                      int32_t *shipped)
{
    const int b = blockIdx.x;
    if (b >= P.n_traj) return;
    const int lane = threadIdx.x;
    const int N = P.N, R = P.R;
    const int64_t t0 = P.traj_off[b], t1 = P.traj_off[b + 1];
    int32_t *xs = state + (int64_t)b * P.K * N;
    const int16_t *rank_b = rank + (int64_t)b * R * N;
    for (int64_t t = t0; t < t1; ++t) {
        int k = P.sku[t], r = P.region[t], q = P.qty[t];
        k = k < 0 ? 0 : (k >= P.K ? P.K - 1 : k); // out-of-range input never indexes memory
        r = r < 0 ? 0 : (r >= P.R ? P.R - 1 : r);
        q = q < 1 ? 1 : q;
        int32_t *xk = xs + (int64_t)k * N;
        const int16_t *rk = rank_b + (int64_t)r * N;
        int a = LOST, xa = 0;
        for (int jb = 0; jb < N; jb += WAVE) {
            const int jj = jb + lane;
            int w = 0, xv = 0;
            if (jj < N) {
                w = rk[jj];
                xv = __hip_atomic_load(&xk[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            const uint64_t m = __ballot(xv > 0);
            if (m) {
                const int l = __ffsll((long long)m) - 1;
                a = __shfl(w, l, WAVE);
                xa = __shfl(xv, l, WAVE);
                break;
            }
        }
        const int sh = a >= 0 ? (q < xa ? q : xa) : 0;
        if (lane == 0) {
            actions[t] = a;
            if (shipped) shipped[t] = sh;
            if (a >= 0)
                __hip_atomic_store(&xk[a], xa - sh, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
    }
}

} // namespace

size_t walk_greedy_lds(int N, int R) { return (size_t)4 * (3 * N + 2 * R) * sizeof(int32_t); }

hipError_t launch_walk_greedy(const Prob &P, const Plan &L, int32_t *final_inv, bool has_init,
                              int grid, hipStream_t st)
{
    hipLaunchKernelGGL(k_walk_greedy, dim3(grid), dim3(256), walk_greedy_lds(P.N, P.R), st, P, L,
                       final_inv, has_init ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_serial_greedy(const Prob &P, const int16_t *rank, int32_t *state,
                                int32_t *actions, int32_t *shipped, hipStream_t st)
{
    hipLaunchKernelGGL(k_serial_greedy, dim3(P.n_traj), dim3(64), 0, st, P, rank, state, actions,
                       shipped);
    return hipGetLastError();
}

} // namespace pk

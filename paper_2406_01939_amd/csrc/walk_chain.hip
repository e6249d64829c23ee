// Greedy walk for a partition given per order (any assignment of steps to processes, such
// as the uniform random partitions of Section 4.1).  Such a process may own several runs
// of one SKU, interleaved with other processes' runs.  Under Algorithm 1 it reaches each
// of them having applied the other processes' cached actions and its own fresh ones, so
// (with the clamp reading of the entry scan) run j of process m starts from
//   max(0, x0 - E_j - D),  D = sum over m's earlier runs of the SKU of
//                              q at the warehouse m chose in this pass - q at the cached one,
// E_j being the cached consumption of every earlier run (the entry scan).  One wave walks
// one process's runs of one SKU (a chain) in order, one order at a time, with the
// inventory, D and the run's consumption held in registers (warehouse w in lane w % 64,
// slot w / 64).  A chain starts at its first run past the SKU's frontier: the runs before
// it kept their actions, which are the ones they would choose again, so they add nothing
// to D.
#include "pk_internal.h"

namespace pk {

namespace {

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v)
{
    for (int d = WAVE / 2; d > 0; d >>= 1) {
        const uint64_t o = __shfl_xor(v, d, WAVE);
        v = o < v ? o : v;
    }
    return v;
}

template <int NW> // warehouse slots per lane: N <= 64 * NW
__global__ __launch_bounds__(256) void k_walk_chain_greedy(Prob P, Plan L, int32_t *final_inv,
                                                           int has_init)
{
    const int wave = uniform(threadIdx.x / WAVE), lane = threadIdx.x % WAVE;
    Ctl *ctl = L.ctl;
    if (ctl->done) return;
    const int N = P.N, R = P.R;
    const int pass = ctl->pass;
    const int32_t *fprev = L.fr[(pass - 1) & 1];
    int32_t *fcur = L.fr[pass & 1];
    const bool all = pass == 1 || L.no_frontier;
    const int n_items = all ? ctl->n_sr : ctl->n_active;
    const bool need_E = pass > 1 || has_init;
    int lcp_b = -1;
    unsigned long long n_orders = 0, n_runs = 0, n_changed = 0, n_bytes = 0;
    const int n_waves = gridDim.x * (blockDim.x / WAVE);
    for (int item = wave * gridDim.x + blockIdx.x; item < n_items; item += n_waves) {
        int s = uniform(all ? item : L.active[item]);
        const int32_t f = all ? FR_ALL : fprev[L.sr_seg[s]];
        if (uniform(L.ch_prevj[s]) > f) continue; // walked with an earlier run of its chain
        int32_t D[NW];
#pragma unroll
        for (int k = 0; k < NW; ++k) D[k] = 0;
        for (;;) {
            const RunDesc d = L.rd[s];
            const int lo = uniform(d.lo), hi = uniform(d.hi), key = uniform(d.key);
            const int g = uniform(d.g), j = uniform(d.j), nsr = uniform(d.nsr);
            const int uidx = uniform(d.uidx);
            const int b = key / P.K;
            const int32_t *x0row = P.x0 + (int64_t)key * N;
            const int32_t *Erow = (need_E && j > 0 && uidx >= 0) ? L.E + (int64_t)uidx * N : nullptr;
            const int32_t *crow = P.cost + (int64_t)b * N * R;
            int32_t x[NW], cons[NW];
#pragma unroll
            for (int k = 0; k < NW; ++k) {
                const int w = k * WAVE + lane;
                int32_t v = 0;
                if (w < N) {
                    v = x0row[w] - (Erow ? Erow[w] : 0) - D[k];
                    v = v > 0 ? v : 0;
                }
                x[k] = v;
                cons[k] = 0;
            }
            bool changed = false;
            int n_chg = 0;
            for (int p = lo; p < hi; ++p) {
                const int r = uniform(L.s_region[p]), q = uniform(L.s_qty[p]);
                const int old = uniform(L.s_alpha[p]);
                // greedy: least (cost, index) among the warehouses with stock
                uint64_t best = ~0ull;
#pragma unroll
                for (int k = 0; k < NW; ++k) {
                    const int w = k * WAVE + lane;
                    if (w < N && x[k] > 0) {
                        const uint32_t c = (uint32_t)crow[(int64_t)w * R + r] ^ 0x80000000u;
                        const uint64_t kv = ((uint64_t)c << 32) | (uint32_t)w;
                        best = kv < best ? kv : best;
                    }
                }
                best = wave_min_u64(best);
                const int a = best == ~0ull ? LOST : uniform((int)(uint32_t)best);
                int sh = 0;
                if (a >= 0) {
                    const int ka = a / WAVE, la = a % WAVE;
                    int xa = 0;
#pragma unroll
                    for (int k = 0; k < NW; ++k)
                        if (k == ka) xa = x[k];
                    sh = __shfl(xa, la, WAVE);
                    sh = sh < q ? sh : q;
                    if (lane == la) {
#pragma unroll
                        for (int k = 0; k < NW; ++k)
                            if (k == ka) {
                                x[k] -= sh;
                                cons[k] += q;
                                D[k] += q;
                            }
                    }
                }
                if (old >= 0 && lane == old % WAVE) {
#pragma unroll
                    for (int k = 0; k < NW; ++k)
                        if (k == old / WAVE) D[k] -= q;
                }
                if (lane == 0) {
                    L.s_alpha[p] = a;
                    L.s_ship[p] = sh;
                }
                if (a != old) {
                    changed = true;
                    ++n_chg;
                }
            }
            int wr = 0;
            if (uidx >= 0) {
#pragma unroll
                for (int k = 0; k < NW; ++k) {
                    const int w = k * WAVE + lane;
                    if (w < N) L.u[(int64_t)uidx * N + w] = cons[k];
                }
                ++wr;
            }
            if (final_inv && j == nsr - 1) {
#pragma unroll
                for (int k = 0; k < NW; ++k) {
                    const int w = k * WAVE + lane;
                    if (w < N) final_inv[(int64_t)key * N + w] = x[k];
                }
                ++wr;
            }
            if (lane == 0) {
                if (changed) {
                    atomicMin(&fcur[g], j);
                    if (b != lcp_b) {
                        if (L.traj_lcp[b] < pass) atomicMax(&L.traj_lcp[b], pass);
                        lcp_b = b;
                    }
                }
                n_orders += hi - lo;
                n_runs += 1;
                n_changed += n_chg;
                n_bytes += 20ull * (hi - lo) + 4ull * N * (1 + (Erow ? 1 : 0) + wr);
            }
            const int nx = uniform(L.ch_next[s]);
            if (nx < 0) break;
            if (nx <= s || nx >= ctl->n_sr) { // links always point forward: never loop
                if (lane == 0) atomicOr(&ctl->error, ERR_NO_PROGRESS);
                break;
            }
            s = nx;
        }
    }
    if (lane == 0 && n_runs) {
        unsigned long long *st = ctl->stat[(blockIdx.x * (blockDim.x / WAVE) + wave) % STAT_SLOTS];
        atomicAdd(&st[ST_ORDERS], n_orders);
        atomicAdd(&st[ST_RUNS], n_runs);
        atomicAdd(&st[ST_CHANGED], n_changed);
        atomicAdd(&st[ST_BYTES], n_bytes);
    }
    walk_finish(ctl, lcp_b >= 0);
}

template <int NW>
void launch_chain_t(const Prob &P, const Plan &L, int32_t *final_inv, int has_init, int grid,
                    hipStream_t st)
{
    hipLaunchKernelGGL(k_walk_chain_greedy<NW>, dim3(grid), dim3(256), 0, st, P, L, final_inv,
                       has_init);
}

} // namespace

hipError_t launch_walk_chain_greedy(const Prob &P, const Plan &L, int32_t *final_inv,
                                    bool has_init, int n_cus, hipStream_t st)
{
    const int nw = (P.N + WAVE - 1) / WAVE;
    const int grid = n_cus * 8;
    const int hi = has_init ? 1 : 0;
    if (nw <= 1) launch_chain_t<1>(P, L, final_inv, hi, grid, st);
    else if (nw <= 2) launch_chain_t<2>(P, L, final_inv, hi, grid, st);
    else if (nw <= 4) launch_chain_t<4>(P, L, final_inv, hi, grid, st);
    else if (nw <= 8) launch_chain_t<8>(P, L, final_inv, hi, grid, st);
    else launch_chain_t<16>(P, L, final_inv, hi, grid, st);
    return hipGetLastError();
}

} // namespace pk

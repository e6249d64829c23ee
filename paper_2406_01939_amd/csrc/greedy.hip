// Greedy policy kernels: the Picard run walk and the serial sweep.
//
// Greedy (Section 3.1, inventory as the constraint): among warehouses with stock, the
// least cost[w][region], lowest index on ties; lost sale iff none has stock.  With
// pos[b][r][w] the position of w in region r's (cost, index) order, the choice is the
// warehouse with stock of least position.  The kernels read
// key[b][r][w] = (pos << S) | w (16-bit keys with S = 8 when N <= 256, else 32-bit keys
// with S = 16): the least key among warehouses with stock names the choice.
#include "pk_internal.h"

namespace pk {

namespace {

constexpr int UNKNOWN = -2;

// Key table layout: per trajectory R rows of npad keys (rows padded to 32 bytes, one
// step of least_key, with all-ones keys, never selected).
template <typename KeyT> __host__ __device__ inline int tab_npad(int N)
{
    constexpr int per = 32 / (int)sizeof(KeyT);
    return (N + per - 1) / per * per;
}
template <typename KeyT> __host__ __device__ inline int64_t tab_stride(int N, int R)
{
    return (int64_t)R * tab_npad<KeyT>(N);
}
template <typename KeyT> __host__ __device__ constexpr int key_shift()
{
    return sizeof(KeyT) == 2 ? 8 : 16;
}

typedef unsigned short pk_u16x2 __attribute__((ext_vector_type(2)));

// Least key among the warehouses in F (bitmask in LDS) for a 16-byte aligned row of
// npad keys; the warehouse it names, or LOST if F is empty.  Each step reads 32 bytes
// of keys with two 16-byte loads, masks the keys of warehouses without stock to
// all-ones and folds them into a packed 16-bit (or 32-bit) minimum.  The loop is
// wave-uniform; lanes with need == false only follow along.
template <typename KeyT>
__device__ __forceinline__ int least_key(const KeyT *row, const uint64_t *F, int npad, bool need)
{
    const uint4 *row4 = (const uint4 *)row;
    constexpr int PER = 16 / (int)sizeof(KeyT); // keys per 16 bytes
    constexpr int STEP = 2 * PER;               // keys per step (divides 64)
    if constexpr (sizeof(KeyT) == 2) {
        pk_u16x2 acc = {0xffff, 0xffff};
        for (int base = 0; base < npad; base += STEP) {
            const uint32_t fb = (uint32_t)(F[base >> 6] >> (base & 63)) & ((1u << STEP) - 1u);
            if (fb == 0) continue; // wave-uniform
            if (need) {
                const uint4 v0 = row4[base / PER], v1 = row4[base / PER + 1];
                const uint32_t d[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const uint32_t two = (fb >> (2 * i)) & 3u;
                    const uint32_t off =
                        ((two & 1u) ? 0u : 0x0000ffffu) | ((two & 2u) ? 0u : 0xffff0000u);
                    const uint32_t m = d[i] | off;
                    pk_u16x2 mv;
                    __builtin_memcpy(&mv, &m, 4);
                    acc = __builtin_elementwise_min(acc, mv);
                }
            }
        }
        const uint32_t best = acc.x < acc.y ? acc.x : acc.y;
        return best == 0xffffu ? LOST : (int)(best & 0xffu);
    } else {
        uint32_t acc = 0xffffffffu;
        for (int base = 0; base < npad; base += STEP) {
            const uint32_t fb = (uint32_t)(F[base >> 6] >> (base & 63)) & ((1u << STEP) - 1u);
            if (fb == 0) continue;
            if (need) {
                const uint4 v0 = row4[base / PER], v1 = row4[base / PER + 1];
                const uint32_t d[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const uint32_t m = ((fb >> i) & 1u) ? d[i] : 0xffffffffu;
                    acc = m < acc ? m : acc;
                }
            }
        }
        return acc == 0xffffffffu ? LOST : (int)(acc & 0xffffu);
    }
}

// One wave walks one run (a process's orders of one SKU) from its entry state, exactly
// as Algorithm 1's process does, 64 orders at a time:
//  * every lane takes the choice its order would get at the chunk's starting state;
//  * the chunk's demand per chosen warehouse is summed in LDS; a warehouse whose demand
//    exceeds its stock empties inside the chunk, and the first order that finds it
//    empty (exclusive prefix of demand >= stock) is the first order whose choice is no
//    longer valid;
//  * all orders before it are exact (stock only falls, so a choice changes only when
//    the chosen warehouse empties); they are committed and the walk resumes there.
// Choices: the wave keeps the set of warehouses with stock as a bitmask F and memoises
// each region's choice; a memo is recomputed (least key over F) only when its warehouse
// has emptied.  For long runs every region's memo is filled up front.
// Orders: the run is read in 64-order chunks into registers, two chunks ahead of use,
// and each chunk is put into a 128-entry ring in LDS when the walk reaches it.  A step
// reads its 64 orders from the ring at any offset, so a partial commit costs no memory
// round trip, and a chunk's loads have at least one whole step to arrive.  The next
// run's descriptor is loaded while the current run is walked.
// The key table of the run's trajectory is read from LDS (one copy per workgroup for a
// single trajectory, one per wave for small tables) or from global memory.
// Per wave LDS: x[N] stock, tot[N] chunk demand, cons[N] run consumption (unclamped, for
// u), bw[R] memo, count of warehouses with stock, F[ceil(N/64)], ring[128] of
// (region, qty, cached action).
template <typename KeyT> __host__ __device__ inline size_t walk_wave_bytes(int N, int R, int mode)
{
    const size_t tb = (size_t)tab_stride<KeyT>(N, R) * sizeof(KeyT);
    const size_t ints = ((size_t)(3 * N + R + 2) * 4 + 15) & ~(size_t)15;
    const size_t f = ((size_t)8 * ((N + 63) / 64) + 15) & ~(size_t)15;
    return (mode == 1 ? tb : 0) + ints + f + 128 * sizeof(int4);
}

template <typename KeyT, int TABMODE> // 0: global table, 1: per-wave LDS, 2: per-WG LDS
__global__ __launch_bounds__(256) void k_walk_greedy(Prob P, Plan L, const KeyT *key_g,
                                                     int32_t *final_inv, int has_init,
                                                     int32_t *sink)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int N = P.N, R = P.R;
    const int nw = (N + 63) / 64;
    const int npad = tab_npad<KeyT>(N);
    const size_t tab_bytes = (size_t)tab_stride<KeyT>(N, R) * sizeof(KeyT);
    const size_t ints_bytes = ((size_t)(3 * N + R + 2) * 4 + 15) & ~(size_t)15;
    const size_t f_bytes = ((size_t)8 * nw + 15) & ~(size_t)15;
    unsigned char *wb = smem + (TABMODE == 2 ? tab_bytes : 0) +
                        wave * walk_wave_bytes<KeyT>(N, R, TABMODE);
    KeyT *wtab = (KeyT *)wb;
    const size_t ints_off = TABMODE == 1 ? tab_bytes : 0;
    int32_t *x = (int32_t *)(wb + ints_off);
    int32_t *tot = x + N;
    int32_t *cons = tot + N;
    int32_t *bw = cons + N;
    int32_t *nfeas = bw + R;
    uint64_t *F = (uint64_t *)(wb + ints_off + ints_bytes);
    int4 *ring = (int4 *)(wb + ints_off + ints_bytes + f_bytes);
    Ctl *ctl = L.ctl;
    if (ctl->done) return;
    if (TABMODE == 2) { // one trajectory: its table, once per workgroup
        const uint4 *src = (const uint4 *)key_g;
        uint4 *dst = (uint4 *)smem;
        const int n16 = (int)(tab_bytes / 16);
        for (int i = threadIdx.x; i < n16; i += blockDim.x) dst[i] = src[i];
        __syncthreads();
    }
    int tab_b = -1;
    const int pass = ctl->pass;
    int32_t *fcur = L.fr[pass & 1];
    // pass 1 (and the no-frontier mode) walks every run; later passes walk the runs past
    // each SKU's frontier, listed by the entry scan
    const bool all = pass == 1 || L.no_frontier;
    const int n_items = all ? ctl->n_sr : ctl->n_active;
    const bool need_E = pass > 1 || has_init;
    int lcp_b = -1; // last trajectory this wave marked as changed in this pass
    unsigned long long n_orders = 0, n_runs = 0, n_changed = 0, n_bytes = 0;

    // static round-robin over the runs (no shared work counter: one hot address)
    const int n_waves = gridDim.x * (blockDim.x / WAVE);
    int item = blockIdx.x * (blockDim.x / WAVE) + wave;
    RunDesc d = {};
    if (item < n_items) d = L.rd[all ? item : L.active[item]];
    for (; item < n_items; item += n_waves) {
        const int lo = d.lo, hi = d.hi, key = d.key, g = d.g, j = d.j, nsr = d.nsr;
        const int uidx = d.uidx;
        const int b = key / P.K;
        const int nxt = item + n_waves;
        const int s_next = nxt < n_items ? (all ? nxt : L.active[nxt]) : -1;
        // the run's first two chunks (loads clamped into the run)
        const int nch = (hi - lo + WAVE - 1) / WAVE;
        int ia = lo + lane < hi ? lo + lane : hi - 1;
        int ra = L.s_region[ia], qa = L.s_qty[ia], oa = L.s_alpha[ia];
        int ib = lo + WAVE + lane < hi ? lo + WAVE + lane : hi - 1;
        int rb = L.s_region[ib], qb = L.s_qty[ib], ob = L.s_alpha[ib];
        const int32_t *x0row = P.x0 + (int64_t)key * N;
        const int32_t *Erow = (need_E && j > 0) ? L.E + (int64_t)uidx * N : nullptr;
        const KeyT *tab;
        if (TABMODE == 0) {
            tab = key_g + b * tab_stride<KeyT>(N, R);
        } else if (TABMODE == 1) {
            if (b != tab_b) { // this wave's copy of the run's trajectory table
                const uint4 *src = (const uint4 *)(key_g + b * tab_stride<KeyT>(N, R));
                uint4 *dst = (uint4 *)wtab;
                const int n16 = (int)(tab_bytes / 16);
                for (int i = lane; i < n16; i += WAVE) dst[i] = src[i];
                tab_b = b;
            }
            tab = wtab;
        } else {
            tab = (const KeyT *)smem;
        }
        int nf = 0;
        for (int k = 0; k < nw; ++k) {
            const int w = k * WAVE + lane;
            int32_t v = 0;
            if (w < N) {
                v = x0row[w] - (Erow ? Erow[w] : 0);
                v = v > 0 ? v : 0;
                x[w] = v;
                tot[w] = 0;
                cons[w] = 0;
            }
            const uint64_t m = __ballot(v > 0);
            if (lane == 0) F[k] = m;
            nf += __popcll(m);
        }
        if (lane == 0) *nfeas = nf;
        ring[lane] = make_int4(ra, qa, oa, 0); // chunk 0
        // next run's descriptor, and chunk 2 into the slot chunk 0 has left
        RunDesc dn = {};
        if (s_next >= 0) dn = L.rd[s_next];
        ia = lo + 2 * WAVE + lane < hi ? lo + 2 * WAVE + lane : hi - 1;
        ra = L.s_region[ia]; qa = L.s_qty[ia]; oa = L.s_alpha[ia];
        int cw = 1; // chunks in the ring
        wave_sync();
        if (hi - lo >= 2 * WAVE) { // long run: every region's choice up front
            for (int rb0 = 0; rb0 < R; rb0 += WAVE) {
                const int rr = rb0 + lane;
                const bool mine = rr < R;
                const int c = least_key<KeyT>(tab + (int64_t)(mine ? rr : 0) * npad, F, npad, mine);
                if (mine) bw[rr] = c;
            }
        } else {
            for (int rr = lane; rr < R; rr += WAVE) bw[rr] = UNKNOWN;
        }
        wave_sync();
        bool changed = false;
        int p = lo;
        while (p < hi) {
            const int off = p - lo;
            // the step reads positions off .. off+63: chunks up to (off + 63) / 64
            const int need_c = (off + WAVE - 1) / WAVE + 1 < nch ? (off + WAVE - 1) / WAVE + 1 : nch;
            if (cw < need_c) { // at most one new chunk per step (a step advances <= 64)
                const int pc = lo + (cw + 2) * WAVE + lane;
                const int ic = pc < hi ? pc : hi - 1;
                if (cw & 1) {
                    ring[WAVE + lane] = make_int4(rb, qb, ob, 0);
                    rb = L.s_region[ic]; qb = L.s_qty[ic]; ob = L.s_alpha[ic];
                } else {
                    ring[lane] = make_int4(ra, qa, oa, 0);
                    ra = L.s_region[ic]; qa = L.s_qty[ic]; oa = L.s_alpha[ic];
                }
                ++cw;
                wave_sync();
            }
            const int n = hi - p < WAVE ? hi - p : WAVE;
            const bool act = lane < n;
            const int4 e = ring[(off + lane) & (2 * WAVE - 1)];
            const int r = act ? e.x : 0, q = act ? e.y : 1, old = e.z;
            int a = LOST;
            if (*nfeas > 0) {
                bool need = false;
                if (act) {
                    a = bw[r];
                    need = a == UNKNOWN || (a >= 0 && !((F[a >> 6] >> (a & 63)) & 1ull));
                }
                if (__ballot(need)) {
                    const int c = least_key<KeyT>(tab + (int64_t)r * npad, F, npad, need);
                    if (need) {
                        a = c;
                        bw[r] = c;
                    }
                }
            }
            wave_sync();
            if (act && a >= 0) atomicAdd(&tot[a], q);
            wave_sync();
            const bool flag = act && a >= 0 && tot[a] > x[a];
            uint64_t todo = __ballot(flag);
            int cut = n;
            int ship = q;
            if (todo) {
                const bool unit = __ballot(act && q != 1) == 0;
                while (todo) {
                    const int l0 = __ffsll((long long)todo) - 1;
                    const int w0 = __builtin_amdgcn_readlane(a, l0);
                    const bool mine = act && a == w0;
                    const uint64_t eq = __ballot(mine);
                    int excl;
                    if (unit) {
                        excl = __popcll(eq & lanemask_lt()); // demand of earlier lanes on w0
                    } else {
                        const int qq = mine ? q : 0;
                        excl = wave_incl_sum(qq) - qq;
                    }
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
            }
            const bool commit = act && lane < cut;
            const bool chg = commit && a != old;
            changed |= chg;
            n_changed += __popcll(__ballot(chg));
            const int sh = a >= 0 ? ship : 0;
            int32_t *pa = commit ? &L.s_alpha[p + lane] : &sink[lane];
            int32_t *ps = commit ? &L.s_ship[p + lane] : &sink[WAVE + lane];
            *pa = a;
            *ps = sh;
            wave_sync();
            bool emptied = false;
            if (commit && a >= 0) {
                const int before = atomicSub(&x[a], ship);
                emptied = before == ship; // this order took the last unit
                atomicAdd(&cons[a], q);
            }
            if (act && a >= 0) tot[a] = 0;
            if (emptied) atomicAnd((unsigned long long *)&F[a >> 6], ~(1ull << (a & 63)));
            const int ne = __popcll(__ballot(emptied));
            if (ne && lane == 0) *nfeas -= ne;
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
                // read first: most changed runs find these already set
                if (b != lcp_b) { // once per trajectory and wave; read first (one hot word)
                    if (L.traj_lcp[b] < pass) atomicMax(&L.traj_lcp[b], pass);
                    lcp_b = b;
                }
            }
            n_orders += hi - lo;
            n_runs += 1;
            n_bytes += 20ull * (hi - lo) + 4ull * N * (1 + (Erow ? 1 : 0) + wr);
        }
        wave_sync();
        d = dn;
    }
    if (lane == 0 && n_runs) {
        unsigned long long *st = ctl->stat[(blockIdx.x * 4 + wave) % STAT_SLOTS];
        atomicAdd(&st[ST_ORDERS], n_orders);
        atomicAdd(&st[ST_RUNS], n_runs);
        atomicAdd(&st[ST_CHANGED], n_changed);
        atomicAdd(&st[ST_BYTES], n_bytes);
    }
    walk_finish(ctl, lcp_b >= 0);
}

// Serial sweep: one wave per trajectory walks its orders in time order.  The stock of
// the trajectory lives in `state` ([K][N], initialised to x0).  Per order, lanes cover
// warehouses: each loads the stock and the region's key of its warehouses (two
// independent loads), the wave takes the least key among warehouses with stock, and
// lane 0 applies f.  The store is fenced before the next order's loads.
template <typename KeyT>
__global__ __launch_bounds__(64) void k_serial_greedy(Prob P, const KeyT *keys, int32_t *state,
                                                      int32_t *actions, int32_t *shipped)
{
    const int b = blockIdx.x;
    if (b >= P.n_traj) return;
    const int lane = threadIdx.x;
    const int N = P.N, R = P.R;
    const int npad = tab_npad<KeyT>(N);
    const int64_t t0 = P.traj_off[b], t1 = P.traj_off[b + 1];
    int32_t *xs = state + (int64_t)b * P.K * N;
    const KeyT *key_b = keys + b * tab_stride<KeyT>(N, R);
    for (int64_t t = t0; t < t1; ++t) {
        int k = P.sku[t], r = P.region[t], q = P.qty[t];
        k = k < 0 ? 0 : (k >= P.K ? P.K - 1 : k); // out-of-range input never indexes memory
        r = r < 0 ? 0 : (r >= P.R ? P.R - 1 : r);
        q = q < 1 ? 1 : q;
        int32_t *xk = xs + (int64_t)k * N;
        const KeyT *kr = key_b + (int64_t)r * npad;
        uint32_t best_l = 0xffffffffu; // least key of a warehouse with stock (this lane)
        int xa_l = 0;
        for (int w = lane; w < N; w += WAVE) {
            const int xv = __hip_atomic_load(&xk[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            const uint32_t kk = (uint32_t)kr[w];
            if (xv > 0 && kk < best_l) { best_l = kk; xa_l = xv; }
        }
        uint32_t best = best_l;
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) {
            const uint32_t o = (uint32_t)__shfl_xor((int)best, d, WAVE);
            best = o < best ? o : best;
        }
        int a = LOST, xa = 0;
        if (best != 0xffffffffu) {
            a = (int)(best & ((1u << key_shift<KeyT>()) - 1u));
            const uint64_t m = __ballot(best_l == best);
            xa = __builtin_amdgcn_readlane(xa_l, __ffsll((long long)m) - 1);
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

// key[b][r][w] = (position of w in region r's increasing (cost[b][w][r], w) order) << S
// | w: one thread per (b, r, w) counts the warehouses that precede w.  Row padding is
// all-ones.
template <typename KeyT>
__global__ void k_keys(Prob P, KeyT *keys)
{
    const int npad = tab_npad<KeyT>(P.N);
    const int64_t n = (int64_t)P.n_traj * P.R * npad;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int w = (int)(i % npad);
        const int64_t br = i / npad;
        const int r = (int)(br % P.R);
        const int b = (int)(br / P.R);
        KeyT *dst = keys + b * tab_stride<KeyT>(P.N, P.R) + (int64_t)r * npad + w;
        if (w >= P.N) {
            *dst = (KeyT)~(KeyT)0;
            continue;
        }
        const int32_t *c = P.cost + (int64_t)b * P.N * P.R;
        const int32_t cw = c[(int64_t)w * P.R + r];
        uint32_t q = 0;
        for (int v = 0; v < P.N; ++v) {
            const int32_t cv = c[(int64_t)v * P.R + r];
            q += (cv < cw) || (cv == cw && v < w);
        }
        *dst = (KeyT)((q << key_shift<KeyT>()) | (uint32_t)w);
    }
}

struct WalkCfg {
    int mode;
    size_t lds;
};

template <typename KeyT> WalkCfg walk_cfg_t(int N, int R, int n_traj)
{
    const size_t tb = (size_t)tab_stride<KeyT>(N, R) * sizeof(KeyT);
    const size_t per = walk_wave_bytes<KeyT>(N, R, 0);
    const size_t per1 = walk_wave_bytes<KeyT>(N, R, 1);
    if (n_traj == 1 && tb + 4 * per <= 64 * 1024) return {2, tb + 4 * per};
    if (tb <= 8 * 1024 && 4 * per1 <= 64 * 1024) return {1, 4 * per1};
    return {0, 4 * per};
}

template <typename KeyT>
void launch_walk_t(const Prob &P, const Plan &L, const void *keys, int32_t *final_inv, int hi,
                   int grid, hipStream_t st)
{
    const WalkCfg c = walk_cfg_t<KeyT>(P.N, P.R, P.n_traj);
    const KeyT *t = (const KeyT *)keys;
    if (c.mode == 2)
        hipLaunchKernelGGL((k_walk_greedy<KeyT, 2>), dim3(grid), dim3(256), c.lds, st, P, L, t,
                           final_inv, hi, L.sink);
    else if (c.mode == 1)
        hipLaunchKernelGGL((k_walk_greedy<KeyT, 1>), dim3(grid), dim3(256), c.lds, st, P, L, t,
                           final_inv, hi, L.sink);
    else
        hipLaunchKernelGGL((k_walk_greedy<KeyT, 0>), dim3(grid), dim3(256), c.lds, st, P, L, t,
                           final_inv, hi, L.sink);
}

} // namespace

bool keys16(int N) { return N <= 256; }

size_t pos_bytes(int N, int R, int n_traj)
{
    return keys16(N) ? (size_t)n_traj * tab_stride<uint16_t>(N, R) * 2
                     : (size_t)n_traj * tab_stride<uint32_t>(N, R) * 4;
}

hipError_t setup_pos(const Prob &P, void *keys, hipStream_t st)
{
    const int64_t n = (int64_t)P.n_traj * P.R * (P.N + 8);
    int64_t g = (n + 255) / 256;
    g = g < 1 ? 1 : (g > 8192 ? 8192 : g);
    if (keys16(P.N))
        hipLaunchKernelGGL(k_keys<uint16_t>, dim3((unsigned)g), dim3(256), 0, st, P, (uint16_t *)keys);
    else
        hipLaunchKernelGGL(k_keys<uint32_t>, dim3((unsigned)g), dim3(256), 0, st, P, (uint32_t *)keys);
    return hipGetLastError();
}

size_t walk_greedy_lds(int N, int R)
{
    return keys16(N) ? walk_cfg_t<uint16_t>(N, R, 2).lds : walk_cfg_t<uint32_t>(N, R, 2).lds;
}

hipError_t launch_walk_greedy(const Prob &P, const Plan &L, const void *keys, int32_t *final_inv,
                              bool has_init, int grid, hipStream_t st)
{
    if (keys16(P.N))
        launch_walk_t<uint16_t>(P, L, keys, final_inv, has_init ? 1 : 0, grid, st);
    else
        launch_walk_t<uint32_t>(P, L, keys, final_inv, has_init ? 1 : 0, grid, st);
    return hipGetLastError();
}

hipError_t launch_serial_greedy(const Prob &P, const void *keys, int32_t *state, int32_t *actions,
                                int32_t *shipped, hipStream_t st)
{
    if (keys16(P.N))
        hipLaunchKernelGGL(k_serial_greedy<uint16_t>, dim3(P.n_traj), dim3(64), 0, st, P,
                           (const uint16_t *)keys, state, actions, shipped);
    else
        hipLaunchKernelGGL(k_serial_greedy<uint32_t>, dim3(P.n_traj), dim3(64), 0, st, P,
                           (const uint32_t *)keys, state, actions, shipped);
    return hipGetLastError();
}

} // namespace pk

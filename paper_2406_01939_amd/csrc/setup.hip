// Per-call setup of the Picard iteration: the partition of the steps into processes.
//
// Each trajectory's orders are sorted (stably) by SKU inside the trajectory's own range, so
// the batch is ordered by key = trajectory * K + SKU and every SKU's orders form a
// contiguous segment in time order.  Blocks of B consecutive sorted positions are the
// processes (Section 2: each process m owns a disjoint set of steps T_m).  A run is a
// block's part of one segment; because SKUs never interact without node capacity
// (Assumption 1, inventory independence), a process's runs are independent and a run is
// the unit of work on the GPU.
//
// The sort key word carries the SKU in its low bits and, when they fit, the order's region
// and quantity above them (the sort looks at the SKU bits only), so the sorted order data
// is read back in sequence instead of gathered through the permutation.
#include <algorithm>
#include <stddef.h>

#include "pk_internal.h"

namespace pk {

namespace {

// Bit fields of a sort key word: SKU in [0, kb), region in [kb, kb + rb), quantity above
// (0 there when the quantity does not fit, which Ctl::qty_unpacked reports).  on: region
// and quantity are packed (kb + rb <= 31).
struct KeyPack {
    int kb, rb, qb;
    int on;
};

KeyPack key_pack(int K, int R)
{
    KeyPack k;
    k.kb = 1;
    while (k.kb < 31 && (1ll << k.kb) < (int64_t)K) ++k.kb;
    k.rb = region_bits(R);
    k.on = k.kb + k.rb <= 31;
    k.qb = k.on ? 32 - k.kb - k.rb : 0;
    return k;
}

__global__ void k_make_keys(Prob P, KeyPack kp, int32_t *keys, int32_t *vals, int validate,
                            Ctl *ctl)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const uint32_t qcap = kp.on ? (uint32_t)((1ull << kp.qb) - 1ull) : 0u;
    int unpacked = 0;
    for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < P.total; o += stride) {
        int32_t s = P.sku[o];
        if (validate) {
            const int32_t r = P.region[o], q = P.qty[o];
            if (s < 0 || s >= P.K || r < 0 || r >= P.R || q < 1) atomicOr(&ctl->error, 1);
        }
        s = s < 0 ? 0 : (s >= P.K ? P.K - 1 : s); // out-of-range input never indexes memory
        uint32_t w = (uint32_t)s;
        if (kp.on) {
            int32_t r = P.region[o], q = P.qty[o];
            r = r < 0 ? 0 : (r >= P.R ? P.R - 1 : r);
            q = q < 1 ? 1 : q;
            uint32_t qw = (uint32_t)q;
            if (qw > qcap) {
                qw = 0;
                unpacked = 1;
            }
            w |= ((uint32_t)r << kp.kb) | (kp.qb > 0 ? qw << (kp.kb + kp.rb) : 0u);
        }
        keys[o] = (int32_t)w;
        vals[o] = (int32_t)o;
    }
    if (__ballot(unpacked) && __lane_id() == 0) atomicOr(&ctl->qty_unpacked, 1);
}

__global__ void k_check_inv(const int32_t *x0, int64_t n, Ctl *ctl)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        if (x0[i] < 0) atomicOr(&ctl->error, 2);
}

// A run starts at every segment start and, inside a segment, where the process changes:
// every B positions for block partitions, where the given process differs for others.
__device__ __forceinline__ bool run_start_at(const Plan &L, int64_t p, bool seg_start)
{
    if (seg_start) return true;
    if (L.worker) return L.worker[L.perm[p]] != L.worker[L.perm[p - 1]];
    return (p % L.B) == 0;
}

// The sorted order data and the run/segment start flags, each workgroup over a contiguous
// range of positions (its trajectory found once, then followed).  Region and quantity come
// from the sorted key words, or through the permutation when they are not packed.
// flags[p] packs the run-start count in the low 32 bits and the segment-start count in the
// high 32 bits.
constexpr int GATHER_PER_WG = 2048;

__global__ __launch_bounds__(256) void k_gather(Prob P, Plan L, KeyPack kp, const int32_t *words,
                                                const int32_t *init_cache, int validate,
                                                int64_t *flags, int want_t)
{
    __shared__ int s_b;
    const int64_t p0 = (int64_t)blockIdx.x * GATHER_PER_WG;
    if (p0 >= P.total) return;
    if (threadIdx.x == 0) s_b = traj_of(P.traj_off, P.n_traj, p0);
    __syncthreads();
    int b = s_b;
    const uint32_t kmask = (uint32_t)((1ull << kp.kb) - 1ull);
    const uint32_t rmask = (uint32_t)((1ull << kp.rb) - 1ull);
    const bool from_words = kp.on && !L.ctl->qty_unpacked;
    const int64_t p1 = p0 + GATHER_PER_WG < P.total ? p0 + GATHER_PER_WG : P.total;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
        while (p >= P.traj_off[b + 1]) ++b; // positions only grow; empty trajectories skipped
        const int32_t o = L.perm[p];
        const uint32_t w = (uint32_t)words[p];
        const int32_t sku = (int32_t)(w & kmask);
        int32_t r, q;
        if (kp.on) {
            r = (int32_t)((w >> kp.kb) & rmask);
            q = from_words ? (int32_t)(w >> (kp.kb + kp.rb)) : P.qty[o];
        } else {
            r = P.region[o];
            q = P.qty[o];
        }
        const int32_t key = b * P.K + sku;
        L.s_key[p] = key;
        r = r < 0 ? 0 : (r >= P.R ? P.R - 1 : r);
        q = q < 1 ? 1 : q;
        L.s_region[p] = r;
        L.s_qty[p] = q;
        if (L.s_rq) { // region | quantity << rq_rb for the first pass's lane walk
            const bool fits = (int64_t)q < (1ll << (31 - L.rq_rb));
            if (!fits) L.ctl->rq_bad = 1;
            L.s_rq[p] = fits ? (int32_t)((uint32_t)r | ((uint32_t)q << L.rq_rb)) : r;
        }
        int32_t a = LOST;
        if (init_cache) {
            a = init_cache[o];
            if (a < LOST || a >= P.N) {
                if (validate) atomicOr(&L.ctl->error, 4);
                a = LOST;
            }
        }
        L.s_alpha[p] = a;
        if (L.worker && L.worker[o] < 0) atomicOr(&L.ctl->error, ERR_PARTITION);
        if (want_t) L.s_t[p] = (int32_t)(o - P.traj_off[b]);
        const bool seg_start = p == P.traj_off[b] || (((uint32_t)words[p - 1]) & kmask) != (uint32_t)sku;
        const bool run_start = run_start_at(L, p, seg_start);
        flags[p] = (run_start ? 1ll : 0ll) | (seg_start ? (1ll << 32) : 0ll);
    }
}

// Run and segment tables from the inclusive scan of the flags.
__global__ void k_tables(Prob P, Plan L, const int64_t *flags)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P.total; p += stride) {
        const int64_t f = flags[p];
        const int32_t sr = (int32_t)(f & 0xffffffffll) - 1;
        const int32_t sg = (int32_t)(f >> 32) - 1;
        const bool seg_start = p == 0 || L.s_key[p - 1] != L.s_key[p];
        const bool run_start = run_start_at(L, p, seg_start);
        if (run_start) {
            L.sr_lo[sr] = (int32_t)p;
            L.sr_seg[sr] = sg;
        }
        if (seg_start) {
            L.seg_key[sg] = L.s_key[p];
            L.seg_sr0[sg] = sr;
        }
        if (p == P.total - 1) {
            L.sr_lo[sr + 1] = (int32_t)P.total;
            L.seg_sr0[sg + 1] = sr + 1;
            L.ctl->n_sr = sr + 1;
            L.ctl->n_seg = sg + 1;
        }
    }
}

// Per segment: (number of runs if split, else 0) | (1 if split) << 32, for one scan.  Also
// initialises the frontiers (pass 1 evaluates everything).
__global__ void k_split_count(Plan L, int64_t *cnt, int32_t n_seg_max)
{
    const int n_seg = L.ctl->n_seg;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_seg_max; g += stride) {
        int64_t c = 0;
        if (g < n_seg) {
            const int32_t nsr = L.seg_sr0[g + 1] - L.seg_sr0[g];
            c = nsr > 1 ? ((int64_t)nsr | (1ll << 32)) : 0;
            L.fr[0][g] = FR_ALL;
            L.fr[1][g] = FR_NONE;
        }
        cnt[g] = c;
    }
}

// Per segment: the list of split segments, and the split counts in the control block.
// base[g]: exclusive prefix over segments of (runs if split) | (1 if split) << 32.
__global__ void k_split_fill(Plan L, const int64_t *base, int32_t n_seg_max)
{
    const int n_seg = L.ctl->n_seg;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_seg; g += stride) {
        const int32_t s0 = L.seg_sr0[g], s1 = L.seg_sr0[g + 1];
        const int32_t ubase = (int32_t)(base[g] & 0xffffffffll), segbase = (int32_t)(base[g] >> 32);
        if (s1 - s0 > 1) L.split_segs[segbase] = (int32_t)g;
        if (g == n_seg - 1) {
            const int32_t last = s1 - s0 > 1 ? s1 - s0 : 0;
            L.ctl->n_split = ubase + last;
            L.ctl->n_split_seg = segbase + (s1 - s0 > 1 ? 1 : 0);
        }
    }
}

// Per run (one thread each): its row of u/E if its segment is split, its place in the
// split list, and its descriptor.
__global__ void k_run_desc(Plan L, const int64_t *base)
{
    const int n_sr = L.ctl->n_sr;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t si = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; si < n_sr; si += stride) {
        const int32_t s = (int32_t)si;
        const int32_t g = L.sr_seg[s];
        const int32_t s0 = L.seg_sr0[g], s1 = L.seg_sr0[g + 1];
        const bool split = s1 - s0 > 1;
        const int32_t uidx = split ? (int32_t)(base[g] & 0xffffffffll) + (s - s0) : -1;
        L.sr_uidx[s] = uidx;
        if (split) L.split_list[uidx] = s;
        L.rd[s] = RunDesc{L.sr_lo[s], L.sr_lo[s + 1], L.seg_key[g], g, s - s0, s1 - s0, uidx, 0};
    }
}

// Chains of a given partition: a process's runs of one segment, in order.  The runs are
// sorted stably by process and then by segment, so each chain's runs become neighbours;
// entries past the run count (keys 0x7fffffff) sort last and are ignored.
__global__ void k_chain_keys(Plan L, int64_t n, int32_t *keys, int32_t *vals)
{
    const int n_sr = L.ctl->n_sr;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += stride) {
        const bool run = s < n_sr;
        keys[s] = run ? L.worker[L.perm[L.sr_lo[s]]] : 0x7fffffff;
        vals[s] = (int32_t)s;
        if (run) {
            L.ch_prevj[s] = -1;
            L.ch_next[s] = -1;
        }
    }
}

__global__ void k_chain_seg_keys(Plan L, int64_t n, const int32_t *vals, int32_t *keys)
{
    const int n_sr = L.ctl->n_sr;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int32_t s = vals[i];
        keys[i] = s < n_sr ? L.sr_seg[s] : 0x7fffffff;
    }
}

// vals: runs in (segment, process, position) order; neighbours of one chain are linked.
__global__ void k_chain_link(Plan L, int64_t n, const int32_t *vals)
{
    const int n_sr = L.ctl->n_sr;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i + 1 < n; i += stride) {
        const int32_t s = vals[i], t = vals[i + 1];
        if (s >= n_sr || t >= n_sr) continue;
        const int32_t g = L.sr_seg[s];
        if (L.sr_seg[t] != g) continue;
        if (L.worker[L.perm[L.sr_lo[s]]] != L.worker[L.perm[L.sr_lo[t]]]) continue;
        L.ch_next[s] = t;
        L.ch_prevj[t] = s - L.seg_sr0[g];
    }
}

// The first pass's run list: key 0 for runs longer than lane_max (the wave-per-run walk's,
// kept in run order by the stable sort), lane_max + 1 - length for the others (longest
// first), 511 past the run count.
__global__ void k_lane_keys(Plan L, int64_t n, int32_t *keys, int32_t *vals)
{
    const int n_sr = L.ctl->n_sr;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += stride) {
        int32_t k = 511;
        if (s < n_sr) {
            const int32_t len = L.sr_lo[s + 1] - L.sr_lo[s];
            k = len > L.lane_max ? 0 : L.lane_max + 1 - len;
        }
        keys[s] = k;
        vals[s] = (int32_t)s;
    }
}

// Splits the sorted list: n_wide = the first position with a nonzero key (binary search).
__global__ void k_lane_count(Plan L, const int32_t *keys)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int n_sr = L.ctl->n_sr;
    int a = 0, b = n_sr; // keys[0, a) are 0, keys[b, n_sr) are not
    while (a < b) {
        const int m = a + (b - a) / 2;
        if (keys[m] == 0) a = m + 1;
        else b = m;
    }
    if (L.ctl->rq_bad) a = n_sr; // a quantity too large for the packed words: no lane walk
    L.ctl->n_wide = a;
    L.ctl->n_lane = n_sr - a;
}

__global__ void k_init_ctl(Ctl *ctl, int32_t *traj_lcp, int n_traj, int max_passes)
{
    // the control block word by word: pass 1, the pass limit, everything else zero
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nthreads = gridDim.x * blockDim.x;
    uint32_t *w = (uint32_t *)ctl;
    const int nw = (int)(sizeof(Ctl) / 4);
    const int i_pass = (int)(offsetof(Ctl, pass) / 4), i_max = (int)(offsetof(Ctl, max_passes) / 4);
    for (int i = tid; i < nw; i += nthreads)
        w[i] = i == i_pass ? 1u : (i == i_max ? (uint32_t)max_passes : 0u);
    for (int b = tid; b < n_traj; b += nthreads) traj_lcp[b] = 0;
}

inline unsigned grid_for(int64_t n, int threads, int cap = 65535)
{
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

} // namespace

// Reset the control block (must precede every other setup step).
hipError_t setup_ctl(Plan &L, int n_traj, int max_passes, hipStream_t st)
{
    const int64_t n = std::max<int64_t>(n_traj, (int64_t)(sizeof(Ctl) / 4));
    hipLaunchKernelGGL(k_init_ctl, dim3(grid_for(n, 256)), dim3(256), 0, st, L.ctl, L.traj_lcp,
                       n_traj, max_passes);
    return hipGetLastError();
}

// The setup scratch: three int32 arrays and an int64 array of `total` entries, then the
// primitives' tmp.
struct ScratchArrays {
    int32_t *keys_a, *keys_b, *vals_b;
    int64_t *flags;
    void *tmp;
};

ScratchArrays scratch_arrays(void *scratch, int64_t n)
{
    char *s = (char *)scratch;
    auto take = [&](size_t bytes) {
        void *r = s;
        s += (bytes + 255) & ~(size_t)255;
        return r;
    };
    ScratchArrays a;
    a.keys_a = (int32_t *)take(n * sizeof(int32_t));
    a.keys_b = (int32_t *)take(n * sizeof(int32_t));
    a.vals_b = (int32_t *)take(n * sizeof(int32_t));
    a.flags = (int64_t *)take(n * sizeof(int64_t));
    a.tmp = s;
    return a;
}

// Sort, gather, and build the run / segment tables.  `scratch` (setup_scratch_bytes) holds
// 3 total int32 (the sort's key words and its second value array), total int64 (flags) and
// the primitives' tmp.
hipError_t setup_plan(const Prob &P, Plan &L, const int32_t *init_cache, int validate,
                      bool want_t, int32_t n_seg_max, void *scratch, hipStream_t st)
{
    hipError_t e;
    const int64_t n = P.total;
    if (n == 0) return hipSuccess;
    const ScratchArrays sa = scratch_arrays(scratch, n);
    int32_t *keys_a = sa.keys_a, *keys_b = sa.keys_b, *vals_b = sa.vals_b;
    int64_t *flags = sa.flags;
    void *tmp = sa.tmp;

    // each trajectory's orders sorted by SKU in place: an even pass count ends in the
    // first pair, so the values start in the permutation array when the count is even
    const KeyPack kp = key_pack(P.K, P.R);
    const bool even = radix_passes(kp.kb) % 2 == 0;
    int32_t *k_in = even ? keys_a : keys_b, *v_in = even ? L.perm : vals_b;
    int32_t *k_alt = even ? keys_b : keys_a, *v_alt = even ? vals_b : L.perm;
    hipLaunchKernelGGL(k_make_keys, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, P, kp, k_in,
                       v_in, validate, L.ctl);
    if (validate) {
        const int64_t nx = (int64_t)P.n_traj * P.K * P.N;
        hipLaunchKernelGGL(k_check_inv, dim3(grid_for(nx, 256, 8192)), dim3(256), 0, st, P.x0,
                           nx, L.ctl);
    }
    bool in_alt = false;
    e = radix_sort_pairs_seg(k_in, v_in, k_alt, v_alt, n, kp.kb, P.traj_off, P.n_traj, tmp, st,
                             &in_alt);
    if (e != hipSuccess) return e;
    const int32_t *words = in_alt ? k_alt : k_in;
    if ((in_alt ? v_alt : v_in) != L.perm) { // not reached with the placement above
        e = hipMemcpyAsync(L.perm, in_alt ? v_alt : v_in, n * sizeof(int32_t),
                           hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_gather, dim3((unsigned)((n + GATHER_PER_WG - 1) / GATHER_PER_WG)),
                       dim3(256), 0, st, P, L, kp, words, init_cache, validate, flags,
                       want_t ? 1 : 0);
    e = scan_i64(flags, n, true, tmp, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tables, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, P, L, flags);
    // split bookkeeping: packed counts per segment -> one exclusive scan (reuses flags:
    // n_seg_max <= total)
    int64_t *cnt = flags;
    hipLaunchKernelGGL(k_split_count, dim3(grid_for(n_seg_max, 256, 8192)), dim3(256), 0, st, L,
                       cnt, n_seg_max);
    e = scan_i64(cnt, n_seg_max, false, tmp, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_split_fill, dim3(grid_for(n_seg_max, 256, 8192)), dim3(256), 0, st, L,
                       cnt, n_seg_max);
    hipLaunchKernelGGL(k_run_desc, dim3(grid_for(n + n_seg_max, 256, 8192)), dim3(256), 0, st, L,
                       cnt);
    if (L.worker) {
        // chains: at most n runs; the scratch above is free again (keys_a/vals_a reuse the
        // flags area, which holds 2n int32)
        int32_t *ka = (int32_t *)flags, *va = ka + n;
        hipLaunchKernelGGL(k_chain_keys, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, L, n,
                           ka, va);
        bool alt = false;
        e = radix_sort_pairs(ka, va, keys_b, vals_b, n, 31, tmp, st, &alt);
        if (e != hipSuccess) return e;
        int32_t *v1 = alt ? vals_b : va;
        int32_t *k2 = alt ? ka : keys_b, *v2 = alt ? va : vals_b; // the free pair
        hipLaunchKernelGGL(k_chain_seg_keys, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, L,
                           n, v1, k2);
        if (v1 != v2) {
            e = hipMemcpyAsync(v2, v1, n * sizeof(int32_t), hipMemcpyDeviceToDevice, st);
            if (e != hipSuccess) return e;
        }
        int seg_bits = 1;
        while (seg_bits < 31 && (1ll << seg_bits) < (int64_t)n_seg_max) ++seg_bits;
        int32_t *k3 = k2 == ka ? keys_b : ka, *v3 = v2 == va ? vals_b : va;
        e = radix_sort_pairs(k2, v2, k3, v3, n, seg_bits, tmp, st, &alt);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_chain_link, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, L, n,
                           alt ? v3 : v2);
    } else if (L.wlist) {
        // the first pass's run list (at most min(n, run bound) runs: every run has an order)
        const int64_t nb = (n + L.B - 1) / L.B;
        const int64_t nl = std::min<int64_t>(n, nb + n_seg_max + 1);
        int32_t *ka = (int32_t *)flags, *kb = keys_b, *va = vals_b;
        hipLaunchKernelGGL(k_lane_keys, dim3(grid_for(nl, 256, 8192)), dim3(256), 0, st, L, nl,
                           ka, va);
        bool alt = false;
        e = radix_sort_pairs(ka, va, kb, L.wlist, nl, 9, tmp, st, &alt);
        if (e != hipSuccess) return e;
        if (!alt) {
            e = hipMemcpyAsync(L.wlist, va, nl * sizeof(int32_t), hipMemcpyDeviceToDevice, st);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k_lane_count, dim3(1), dim3(64), 0, st, L, alt ? kb : ka);
    }
    return hipGetLastError();
}

// Actions and units shipped back to time order, once per call.  Within each trajectory's
// range the sorted position p holds time index perm[p]; with trajectories of at most 2^20
// orders and N < 4095 the inverse permutation runs as a sort by destination tile and a
// placement through LDS (both coalesced), else as one scattered write per element.
hipError_t unpermute_results(const Prob &P, const Plan &L, int32_t *actions, int32_t *shipped,
                             void *scratch, bool tiles, hipStream_t st)
{
    const int64_t n = P.total;
    if (!tiles || n < 2) return launch_unpermute(P, L, actions, shipped, st);
    const ScratchArrays sa = scratch_arrays(scratch, n);
    int32_t *f = (int32_t *)sa.flags; // 2n int32
    return unpermute_seg(L.perm, L.s_alpha, shipped ? L.s_ship : nullptr, n, P.traj_off,
                         P.n_traj, actions, shipped, sa.keys_a, sa.keys_b, sa.vals_b, f,
                         sa.tmp, st);
}

int region_bits(int R)
{
    int b = 1;
    while (b < 31 && (1ll << b) < (int64_t)R) ++b;
    return b;
}

size_t setup_scratch_bytes(int64_t n, int n_traj)
{
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t t = std::max(radix_tmp_bytes(n, n_traj), scan_tmp_bytes(n));
    return al(n * 4) * 3 + al(n * 8) + al(t) + 1024;
}

} // namespace pk

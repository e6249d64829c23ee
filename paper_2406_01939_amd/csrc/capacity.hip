// Picard iteration with node capacity (Section 3: the FO state is (x_t, c_t); an order of
// SKU i may go to node j only while c_{t,j} > 0 and x_{t,i,j} > 0; shipping one unit lowers
// both).  Unit demand, one trajectory; the greedy policy (least cost, lowest index on ties),
// the capacity-dependent policy of the appendix's ablation or a bid-price policy
// (cap_choose).  Nothing below but the key table and the walk depends on the policy.
//
// Capacity couples the SKUs, so processes are blocks of B consecutive orders in time.
// Under Algorithm 1, process m replays the cached actions of every order before its block
// and nothing after its block reaches it, so it starts from the replay's state at mB.
// That state is computed per pass without a serial replay:
//  * stock: a cached action whose node has no stock ships nothing, so the replayed stock
//    of (SKU k, node w) at mB is max(0, x0[k][w] - n), n = the cached actions of SKU k to
//    w before mB (the clamp composes: max(0, max(0, x - a) - b) = max(0, x - a - b));
//    node capacity is not needed here: once a node's capacity is gone in the replay, its
//    stock no longer matters to any decision (the node is infeasible for every process
//    that starts after that point);
//  * capacity: before node w runs out, a cached action to w ships iff the clamp above
//    passes, so the capacity at mB is max(0, cap0[w] - O_w(mB)), O_w(mB) = the cached
//    actions before mB that pass their stock test, counted per block and scanned.
// The pass:
//  1. k_cap_piece_count / k_cap_piece_scan: cached action counts per (SKU piece, node),
//     scanned along each SKU (pieces cut long SKU segments for parallelism);
//  2. k_cap_entry: one wave per piece takes its positions of the SKU-sorted list 64 at
//     a time, with one lane mask per node; at the first order of each (block, SKU) it
//     writes that block's stock row of the SKU (clamped to 255: a block walk takes at most
//     B <= 255 units from it), and it marks each cached action that passes its stock test
//     (P); after pass 1 only SKUs with a changed order are revisited (cap_sku_stale);
//  3. k_cap_hist, k_cap_scan: per block, the passing actions per node (H); per node, an
//     exclusive scan of H over blocks -> entry capacities;
//  4. k_cap_walk: one wave per block walks its orders in time order with fresh
//     decisions, stock rows in LDS, capacities in registers; only blocks after the first
//     block that changed in the previous pass are walked (an earlier block's inputs did
//     not change, so neither does its output: the paper's reset point).
// The pass with no change ends the iteration.
#include <algorithm>
#include <climits>

#include "pk_internal.h"

namespace pk {

namespace {

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Least of the 64 lanes' values, by DPP: row minima (row_shr 1, 2, 4, 8), then rows 0-1
// and 2-3 (row_bcast 15), then all four (row_bcast 31) in lane 63, read from there.
// Lanes a step does not reach keep the identity CAP_NONE.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v)
{
#define PK_CAP_MIN_DPP(ctrl, rmask)                                                              \
    {                                                                                            \
        const uint32_t o = (uint32_t)__builtin_amdgcn_update_dpp((int)CAP_NONE, (int)v, ctrl,   \
                                                                 rmask, 0xf, false);             \
        v = o < v ? o : v;                                                                       \
    }
    PK_CAP_MIN_DPP(0x111, 0xf) // row_shr:1
    PK_CAP_MIN_DPP(0x112, 0xf) // row_shr:2
    PK_CAP_MIN_DPP(0x114, 0xf) // row_shr:4
    PK_CAP_MIN_DPP(0x118, 0xf) // row_shr:8
    PK_CAP_MIN_DPP(0x142, 0xa) // row_bcast:15 into rows 1 and 3
    PK_CAP_MIN_DPP(0x143, 0xc) // row_bcast:31 into rows 2 and 3
#undef PK_CAP_MIN_DPP
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v)
{
#define PK_CAP_MAX_DPP(ctrl, rmask)                                                              \
    {                                                                                            \
        const uint32_t o = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, ctrl, rmask, 0xf,    \
                                                                 false);                         \
        v = o > v ? o : v;                                                                       \
    }
    PK_CAP_MAX_DPP(0x111, 0xf)
    PK_CAP_MAX_DPP(0x112, 0xf)
    PK_CAP_MAX_DPP(0x114, 0xf)
    PK_CAP_MAX_DPP(0x118, 0xf)
    PK_CAP_MAX_DPP(0x142, 0xa)
    PK_CAP_MAX_DPP(0x143, 0xc)
#undef PK_CAP_MAX_DPP
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v)
{
    for (int d = WAVE / 2; d > 0; d >>= 1) {
        const uint64_t o = __shfl_xor(v, d, WAVE);
        v = o < v ? o : v;
    }
    return v;
}

// The policy's choice for one order, lane l holding nodes 2l and 2l+1: f0/f1 whether each
// has stock and capacity, c0/c1 their capacities, kc their entries of the region's row of
// the key table, bi their bid prices of the order's SKU (CAP_BID only).
//  * CAP_GREEDY: kc = (cost << 8) | w; the least key wins (lowest index on ties);
//  * CAP_GAMMA (the appendix's ablation, gamma = gnum / gden): kc = the node's rank in the
//    region's (cost, index) order; the least
//      gden rank M + gnum (N-1) p(c)
//    wins, lowest index on ties (rank + gamma (N-1) p(c) / M times gden M > 0, in 64 bits),
//    with glow = 0: M = the largest capacity of any node and p(c) = M - c; glow > 0:
//    M = glow and p(c) = max(0, glow - c), a price only near exhaustion;
//  * CAP_BID (fixed dual prices, Section 4.2's dual policy): kc = cost + bid_cap[w]; the
//    least kc + bid_inv[sku][w] (below 2^26) wins, lowest index on ties.
// Returns the node or LOST (wave-uniform).
template <int POL>
__device__ __forceinline__ int cap_choose(uint2 kc, uint2 bi, bool f0, bool f1, int c0, int c1,
                                          int lane, int nm1, int gnum, int gden, int glow)
{
    if constexpr (POL == CAP_GREEDY) {
        const uint32_t ka = f0 ? kc.x : CAP_NONE, kb = f1 ? kc.y : CAP_NONE;
        const uint32_t best = wave_min_u32(ka < kb ? ka : kb);
        return best == CAP_NONE ? LOST : (int)(best & 0xffu);
    } else if constexpr (POL == CAP_BID) {
        const uint64_t none = ~0ull;
        const uint64_t ka = f0 ? (((uint64_t)(kc.x + bi.x) << 8) | (uint64_t)(2 * lane)) : none;
        const uint64_t kb = f1 ? (((uint64_t)(kc.y + bi.y) << 8) | (uint64_t)(2 * lane + 1)) : none;
        const uint64_t best = wave_min_u64(ka < kb ? ka : kb);
        return best == none ? LOST : (int)(best & 0xffu);
    } else {
        const uint64_t M = glow > 0 ? (uint64_t)glow : wave_max_u32((uint32_t)max(max(c0, c1), 0));
        const uint64_t p0 = glow > 0 ? (c0 < glow ? (uint64_t)(glow - c0) : 0ull) : M - (uint64_t)c0;
        const uint64_t p1 = glow > 0 ? (c1 < glow ? (uint64_t)(glow - c1) : 0ull) : M - (uint64_t)c1;
        const uint64_t none = ~0ull;
        const uint64_t ka = f0 ? ((((uint64_t)gden * kc.x * M + (uint64_t)gnum * nm1 * p0) << 8) |
                                  (uint64_t)(2 * lane))
                               : none;
        const uint64_t kb = f1 ? ((((uint64_t)gden * kc.y * M + (uint64_t)gnum * nm1 * p1) << 8) |
                                  (uint64_t)(2 * lane + 1))
                               : none;
        const uint64_t best = wave_min_u64(ka < kb ? ka : kb);
        return best == none ? LOST : (int)(best & 0xffu);
    }
}

// The bid prices of SKU k's stock at this lane's two nodes (zero without bid_inv).
__device__ __forceinline__ uint2 bid_row(const CapPlan &L, int k, int lane)
{
    if (!L.bid_inv) return make_uint2(0u, 0u);
    const int32_t *row = L.bid_inv + (int64_t)k * L.N;
    return make_uint2(2 * lane < L.N ? (uint32_t)row[2 * lane] : 0u,
                      2 * lane + 1 < L.N ? (uint32_t)row[2 * lane + 1] : 0u);
}

__device__ __forceinline__ uint8_t clamp255(int v) { return (uint8_t)(v < 0 ? 0 : (v > 255 ? 255 : v)); }

// ---------------------------------------------------------------- setup
__global__ void k_cap_check(CapPlan L, int64_t n_x0, const int32_t *init)
{
    int32_t err = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < L.T; i += stride) {
        if (L.qty[i] != 1) err |= CAP_ERR_QTY;
        if (L.sku[i] < 0 || L.sku[i] >= L.K) err |= CAP_ERR_SKU;
        if (L.region[i] < 0 || L.region[i] >= L.R) err |= CAP_ERR_REGION;
        if (init && (init[i] < LOST || init[i] >= L.N)) err |= CAP_ERR_INIT;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_x0; i += stride)
        if (L.x0[i] < 0) err |= CAP_ERR_X0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < L.N; i += stride)
        if (L.cap0[i] < 0) err |= CAP_ERR_CAP;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)L.N * L.R;
         i += stride)
        if (L.cost[i] < 0 || L.cost[i] >= (1 << 24)) err |= CAP_ERR_COST;
    if (L.bid_inv)
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_x0; i += stride)
            if (L.bid_inv[i] < 0 || L.bid_inv[i] >= (1 << 24)) err |= CAP_ERR_BID;
    if (L.bid_cap)
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < L.N; i += stride)
            if (L.bid_cap[i] < 0 || L.bid_cap[i] >= (1 << 24)) err |= CAP_ERR_BID;
    if (err) atomicOr(&L.ctl->error, err);
}

__global__ void k_cap_keys(CapPlan L, int32_t *keys, int32_t *vals)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < L.T; t += stride) {
        keys[t] = L.sku[t];
        vals[t] = (int32_t)t;
    }
}

// seg_off[k] = first sorted position whose SKU is >= k, for k = 0..K: position i writes
// the SKUs in (key[i-1], key[i]] (key[-1] = -1, key[T] = K), which covers each k once.
__global__ void k_cap_seg_bounds(CapPlan L, const int32_t *skey)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= L.T; i += stride) {
        const int prev = i > 0 ? skey[i - 1] : -1;
        const int cur = i < L.T ? skey[i] : L.K;
        for (int k = prev + 1; k <= cur; ++k) L.seg_off[k] = (int32_t)i;
    }
}

// Key table, region-major, one 512-byte row per region: greedy keys (cost << 8) | w, for
// the capacity-dependent policy each node's rank in the region's (cost, index) order, for
// bid prices cost + bid_cap[w].
__global__ void k_cap_keytab(CapPlan L)
{
    const int64_t n = (int64_t)L.R * CAP_NPAD;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int r = (int)(i / CAP_NPAD), w = (int)(i % CAP_NPAD);
        if (w >= L.N) {
            L.keyT[i] = CAP_NONE;
        } else if (L.pol == CAP_GREEDY) {
            L.keyT[i] = ((uint32_t)L.cost[(int64_t)w * L.R + r] << 8) | (uint32_t)w;
        } else if (L.pol == CAP_BID) {
            L.keyT[i] = (uint32_t)L.cost[(int64_t)w * L.R + r] +
                        (L.bid_cap ? (uint32_t)L.bid_cap[w] : 0u);
        } else { // rank of w in the region's (cost, index) order
            const int32_t cw = L.cost[(int64_t)w * L.R + r];
            uint32_t k = 0;
            for (int v = 0; v < L.N; ++v) {
                const int32_t cv = L.cost[(int64_t)v * L.R + r];
                k += cv < cw || (cv == cw && v < w);
            }
            L.keyT[i] = k;
        }
    }
}

// One wave per block: a 0/1 flag for the first order of each (block, SKU) (scanned into
// row ids afterwards) and each order's slot, the rank of its SKU's first order among the
// block's first orders (the stock row it uses in the walk's LDS).  The largest number of
// distinct SKUs in a block sizes the walk's LDS.
__global__ __launch_bounds__(64) void k_cap_slots(CapPlan L, int32_t *first)
{
    __shared__ int32_t sk[CAP_MAX_B], fo[CAP_MAX_B];
    const int m = blockIdx.x, lane = threadIdx.x;
    const int lo = m * L.B, hi = min(lo + L.B, L.T), n = hi - lo;
    for (int j = lane; j < n; j += WAVE) sk[j] = L.sku[lo + j];
    __syncthreads();
    for (int j = lane; j < n; j += WAVE) {
        int f = j;
        for (int i = 0; i < j; ++i)
            if (sk[i] == sk[j]) { f = i; break; }
        fo[j] = f;
        first[lo + j] = f == j;
    }
    __syncthreads();
    int nd = 0;
    for (int j = lane; j < n; j += WAVE) {
        const int f = fo[j];
        int c = 0;
        for (int i = 0; i < f; ++i) c += fo[i] == i;
        L.slot[lo + j] = c;
        nd += f == j;
    }
    nd = wave_sum(nd);
    if (lane == 0) atomicMax(&L.ctl->max_distinct, nd);
}

// Pieces of each SKU's segment: ceil(len / CAP_PIECE) of them.
__global__ void k_cap_piece_counts(CapPlan L, int32_t *cnt)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k <= L.K; k += stride) {
        if (k == L.K) { cnt[k] = 0; continue; }
        const int len = L.seg_off[k + 1] - L.seg_off[k];
        cnt[k] = (len + CAP_PIECE - 1) / CAP_PIECE;
    }
}

// One descriptor per piece: SKU, sorted range and whether its SKU has several pieces.
__global__ void k_cap_piece_fill(CapPlan L)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < L.K; k += stride) {
        const int p0 = L.piece_off[k], p1 = L.piece_off[k + 1];
        const int s0 = L.seg_off[k], s1 = L.seg_off[k + 1];
        for (int p = p0; p < p1; ++p) {
            const int lo = s0 + (p - p0) * CAP_PIECE;
            L.piece[p] = make_int4((int)k, lo, min(lo + CAP_PIECE, s1), p1 - p0 > 1);
        }
        if (k == L.K - 1) L.ctl->n_pieces = L.piece_off[L.K];
    }
}

// ---------------------------------------------------------------- one pass
// A SKU's stock rows, pass flags and piece counts depend on its own cached actions only:
// after pass 1 they are rebuilt only for SKUs with an order whose action changed in the
// previous pass (the others keep last pass's values, which are those of their unchanged
// actions; frontier blocks only ever move forward, so no row they need was skipped).
__device__ __forceinline__ bool cap_sku_stale(const CapPlan &L, int k, int pass)
{
    return pass == 1 || L.skuchg[k] == pass - 1;
}

// Cached action counts per piece of the SKUs with more than one piece.
__global__ __launch_bounds__(256) void k_cap_piece_count(CapPlan L)
{
    __shared__ int32_t u[4][CAP_NPAD];
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int n_pieces = L.ctl->n_pieces, pass = L.ctl->pass;
    for (int p = uni(blockIdx.x * 4 + wave); p < n_pieces; p += gridDim.x * 4) {
        const int4 pd = L.piece[p]; // SKU, lo, hi, several pieces
        const int lo = pd.y, hi = pd.z;
        if (!pd.w || !cap_sku_stale(L, pd.x, pass)) continue;
        u[wave][lane] = 0;
        u[wave][WAVE + lane] = 0;
        wave_sync();
        for (int i = lo + lane; i < hi; i += WAVE) {
            const int a = L.alpha[L.perm[i]];
            if (a >= 0) atomicAdd(&u[wave][a], 1);
        }
        wave_sync();
        int32_t *dst = L.pc + (int64_t)p * CAP_NPAD;
        dst[lane] = u[wave][lane];
        dst[WAVE + lane] = u[wave][WAVE + lane];
        wave_sync();
    }
}

// Exclusive scan of the piece counts along each SKU with more than one piece: one
// workgroup per SKU, its four waves taking consecutive quarters of the SKU's pieces
// (quarter sums, then each quarter's offset from the earlier ones, then its prefixes).
__device__ __forceinline__ void pc_sum(const CapPlan &L, int q0, int q1, int lane, int &s0,
                                       int &s1)
{
    constexpr int U = 8; // rows loaded together
    s0 = s1 = 0;
    for (int pb = q0; pb < q1; pb += U) {
        int v0[U], v1[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int32_t *row = L.pc + (int64_t)min(pb + q, q1 - 1) * CAP_NPAD;
            v0[q] = row[lane];
            v1[q] = row[WAVE + lane];
        }
#pragma unroll
        for (int q = 0; q < U; ++q)
            if (pb + q < q1) {
                s0 += v0[q];
                s1 += v1[q];
            }
    }
}

__global__ __launch_bounds__(256) void k_cap_piece_scan(CapPlan L)
{
    __shared__ int32_t qs[4][CAP_NPAD];
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int pass = L.ctl->pass;
    for (int k = blockIdx.x; k < L.K; k += gridDim.x) { // uniform per workgroup
        const int p0 = L.piece_off[k], p1 = L.piece_off[k + 1];
        if (p1 - p0 < 2 || !cap_sku_stale(L, k, pass)) continue;
        const int per = (p1 - p0 + 3) / 4;
        const int q0 = min(p0 + wave * per, p1), q1 = min(q0 + per, p1);
        int s0, s1;
        pc_sum(L, q0, q1, lane, s0, s1);
        qs[wave][lane] = s0;
        qs[wave][WAVE + lane] = s1;
        __syncthreads();
        int run0 = 0, run1 = 0;
        for (int v = 0; v < wave; ++v) {
            run0 += qs[v][lane];
            run1 += qs[v][WAVE + lane];
        }
        constexpr int U = 8; // rows loaded together, then rewritten
        for (int pb = q0; pb < q1; pb += U) {
            int v0[U], v1[U];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const int32_t *row = L.pc + (int64_t)min(pb + q, q1 - 1) * CAP_NPAD;
                v0[q] = row[lane];
                v1[q] = row[WAVE + lane];
            }
#pragma unroll
            for (int q = 0; q < U; ++q) {
                if (pb + q < q1) {
                    int32_t *row = L.pc + (int64_t)(pb + q) * CAP_NPAD;
                    row[lane] = run0;
                    row[WAVE + lane] = run1;
                    run0 += v0[q];
                    run1 += v1[q];
                }
            }
        }
        __syncthreads(); // qs is reused by the next SKU
    }
}

// The SKU-sorted position i of a piece: its order's time, cached action and, for the
// first order of a (block, SKU), the row of X it starts (else -1).
struct CapEnt {
    int t, a, row;
};

__device__ __forceinline__ CapEnt cap_ent(const CapPlan &L, int i, int hi)
{
    CapEnt e = {0, LOST, -1};
    if (i < hi) {
        e.t = L.perm[i];
        e.row = L.srow[i];
        e.a = L.alpha[e.t];
    }
    return e;
}

// Row of X started at each sorted position (-1 unless the position's order is the first
// of its (block, SKU)), in sorted order so that the entry stage reads it coalesced.
__global__ void k_cap_srow(CapPlan L)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < L.T; i += stride) {
        const int t = L.perm[i];
        L.srow[i] = L.first[t] ? L.sid[t] : -1;
    }
}

// One wave per piece: stock rows at each (block, SKU)'s first order and the pass flag of
// every cached action.  Lane l holds nodes l and 64 + l: their stock and the SKU's cached
// actions to them before the current chunk (ca, cb), in registers.  Positions come 64 at
// a time (the next chunk loaded while the current one is used); per chunk, each node's
// lanes form a 64-bit mask (one ballot per distinct node in the chunk), and every count
// the chunk needs is a popcount of a mask below a lane:
//  * the action of lane i to node a is the SKU's (c_a + popc(mask_a below i))-th to a and
//    ships iff that is below the SKU's initial stock at a (the clamp);
//  * the stock row starting at lane i is max(0, x0 - c - popc(mask below i)) per node.
__device__ __forceinline__ void cap_entry_piece(const CapPlan &L, int p, int lane, int pass,
                                                int frontier);

__global__ __launch_bounds__(256) void k_cap_entry(CapPlan L)
{
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int n_pieces = L.ctl->n_pieces, pass = L.ctl->pass;
    const int frontier = L.ctl->frontier;
    for (int p = uni(blockIdx.x * 4 + wave); p < n_pieces; p += gridDim.x * 4)
        cap_entry_piece(L, p, lane, pass, frontier);
}

__device__ __forceinline__ void cap_entry_piece(const CapPlan &L, int p, int lane, int pass,
                                                int frontier)
{
    const int4 pd = L.piece[p]; // SKU, lo, hi, several pieces
    const int k = pd.x, lo = pd.y, hi = pd.z;
    if (!cap_sku_stale(L, k, pass)) return;
    const int N = L.N, B = L.B;
    const int w0 = lane, w1 = WAVE + lane;
    const int x0a = w0 < N ? L.x0[(int64_t)k * N + w0] : 0;
    const int x0b = w1 < N ? L.x0[(int64_t)k * N + w1] : 0;
    int ca = 0, cb = 0;
    if (pd.w) {
        const int32_t *row = L.pc + (int64_t)p * CAP_NPAD;
        ca = row[w0];
        cb = row[w1];
    }
    const uint64_t below = lanemask_lt();
    CapEnt e = cap_ent(L, lo + lane, hi);
    for (int base = lo; base < hi; base += WAVE) {
        const CapEnt nx = cap_ent(L, base + WAVE + lane, hi);
        const bool valid = base + lane < hi;
        const bool act = valid && e.a >= 0;
        // each node's lanes in this chunk
        uint64_t m0 = 0, m1 = 0;
        uint64_t rem = __ballot(act);
        while (rem) {
            const int q = __ffsll((long long)rem) - 1;
            const int v = uni(__shfl(e.a, q, WAVE));
            const uint64_t mv = __ballot(act && e.a == v);
            if (lane == (v & (WAVE - 1))) {
                if (v < WAVE) m0 = mv;
                else m1 = mv;
            }
            rem &= ~mv;
        }
        // pass flags: the owner lane of each action's node supplies its mask, count, stock
        // (every lane takes part in every shuffle: a lane reads only from active lanes)
        const int ol = act ? (e.a & (WAVE - 1)) : 0;
        const bool hiw = e.a >= WAVE;
        const uint64_t ma0 = __shfl(m0, ol, WAVE), ma1 = __shfl(m1, ol, WAVE);
        const int cn0 = __shfl(ca, ol, WAVE), cn1 = __shfl(cb, ol, WAVE);
        const int st0 = __shfl(x0a, ol, WAVE), st1 = __shfl(x0b, ol, WAVE);
        const uint64_t ma = hiw ? ma1 : ma0;
        const int cnt = hiw ? cn1 : cn0, stock = hiw ? st1 : st0;
        if (act) L.P[e.t] = cnt + __popcll(ma & below) < stock;
        // stock rows of the (block, SKU)s that start in this chunk (walked blocks only)
        const bool starts = valid && e.row >= 0 && e.t / B > frontier;
        uint64_t rs = __ballot(starts);
        while (rs) {
            const int i = __ffsll((long long)rs) - 1;
            const int row = uni(__shfl(e.row, i, WAVE));
            const uint64_t bi = (1ull << i) - 1;
            uint8_t *xr = L.X + (int64_t)row * CAP_NPAD;
            xr[w0] = clamp255(x0a - ca - __popcll(m0 & bi));
            xr[w1] = clamp255(x0b - cb - __popcll(m1 & bi));
            rs &= rs - 1;
        }
        ca += __popcll(m0);
        cb += __popcll(m1);
        e = nx;
    }
}

// Passing cached actions per (node, block): one wave per block of orders, counts in LDS.
__global__ __launch_bounds__(256) void k_cap_hist(CapPlan L)
{
    __shared__ int32_t u[4][CAP_NPAD];
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int m = uni(blockIdx.x * 4 + wave);
    // after a pass without change nothing moves (no cached action changed)
    if (m >= L.nblk || L.ctl->frontier == INT_MAX) return;
    u[wave][lane] = 0;
    u[wave][WAVE + lane] = 0;
    wave_sync();
    const int lo = m * L.B, hi = min(lo + L.B, L.T);
    for (int t = lo + lane; t < hi; t += WAVE) {
        const int a = L.alpha[t];
        if (a >= 0 && L.P[t]) atomicAdd(&u[wave][a], 1);
    }
    wave_sync();
    const int64_t nblk = L.nblk;
    if (lane < L.N) L.H[lane * nblk + m] = u[wave][lane];
    if (WAVE + lane < L.N) L.H[(WAVE + lane) * nblk + m] = u[wave][WAVE + lane];
}

// Per node, exclusive scan of the passing counts over blocks: capacity at each block's
// start.
constexpr int CAP_SCAN_T = 1024; // threads per node's scan

__global__ __launch_bounds__(CAP_SCAN_T) void k_cap_scan(CapPlan L)
{
    __shared__ int32_t part[CAP_SCAN_T];
    const int w = blockIdx.x, tid = threadIdx.x;
    if (L.ctl->frontier == INT_MAX) return; // after a pass without change H is unchanged
    const int nblk = L.nblk;
    const int per = (nblk + CAP_SCAN_T - 1) / CAP_SCAN_T;
    const int b0 = tid * per, b1 = min(b0 + per, nblk);
    int32_t *h = L.H + (int64_t)w * nblk;
    int s = 0;
    for (int b = b0; b < b1; ++b) s += h[b];
    part[tid] = s;
    __syncthreads();
    for (int d = 1; d < CAP_SCAN_T; d <<= 1) {
        const int v = tid >= d ? part[tid - d] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int run = tid > 0 ? part[tid - 1] : 0;
    const int c0 = L.cap0[w];
    for (int b = b0; b < b1; ++b) {
        const int v = h[b];
        L.capE[(int64_t)w * nblk + b] = max(0, c0 - run);
        run += v;
    }
}

// One wave per block: the block's orders in time order with fresh greedy decisions.
// Lane l holds nodes 2l and 2l+1 (stock bytes as one 16-bit LDS word, capacities and keys
// in registers).  A lane writes only its own stock word, so steps need no barrier.  The
// block's regions and stock-row slots (and SKUs, for bid prices) sit in registers (order j
// in lane j % 64 of register j / 64) and are read with readlane; each order's keys (and
// bid prices) are loaded four orders ahead.
template <int POL>
__global__ __launch_bounds__(64) void k_cap_walk(CapPlan L)
{
    extern __shared__ __align__(16) unsigned char cap_smem[];
    const int m = blockIdx.x, lane = threadIdx.x;
    CapCtl *ctl = L.ctl;
    if (m <= ctl->frontier) return;
    const int B = L.B;
    const int lo = m * B, hi = min(lo + B, L.T), n = hi - lo;
    const int D = L.dmax; // stock rows per block (the most distinct SKUs of any block)
    uint16_t *rows = (uint16_t *)cap_smem;                       // [D][64] stock words
    int32_t *sd = (int32_t *)(cap_smem + (size_t)D * CAP_NPAD); // [D] row of X per slot
    int32_t *out = sd + D;                                       // [B]
    int rg[4], sv[4]; // regions and slots of orders lane, 64 + lane, 128 + lane, 192 + lane
    int sk[4];        // their SKUs (bid prices only)
    int nd = 0;       // distinct SKUs of this block
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int j = q * WAVE + lane;
        rg[q] = sv[q] = sk[q] = 0;
        if (j < n) {
            rg[q] = L.region[lo + j];
            sv[q] = L.slot[lo + j];
            if constexpr (POL == CAP_BID) sk[q] = L.sku[lo + j];
            if (L.first[lo + j]) {
                sd[sv[q]] = L.sid[lo + j];
                ++nd;
            }
        }
    }
    nd = wave_sum(nd);
    __syncthreads();
    // stock rows of the block's SKUs: 16-byte pieces spread over the lanes, every load of a
    // round issued before its stores
    {
        const uint4 *X4 = (const uint4 *)L.X;
        uint4 *R4 = (uint4 *)rows;
        const int n16 = nd * (CAP_NPAD / 16);
        for (int b0 = 0; b0 < n16; b0 += 4 * WAVE) {
            int r[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int idx = b0 + q * WAVE + lane;
                r[q] = idx < n16 ? sd[idx >> 3] : -1;
            }
            uint4 v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int idx = b0 + q * WAVE + lane;
                v[q] = X4[(int64_t)(r[q] >= 0 ? r[q] : 0) * (CAP_NPAD / 16) + (idx & 7)];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (r[q] >= 0) R4[b0 + q * WAVE + lane] = v[q];
        }
    }
    const int nblk = L.nblk;
    int c0 = 2 * lane < L.N ? L.capE[(int64_t)(2 * lane) * nblk + m] : 0;
    int c1 = 2 * lane + 1 < L.N ? L.capE[(int64_t)(2 * lane + 1) * nblk + m] : 0;
    __syncthreads();
    const uint2 *K2 = (const uint2 *)L.keyT;
    auto lane_val = [&](const int (&a)[4], int j) { // wave-uniform j < 256
        const int q = j >> 6, l = j & (WAVE - 1);
        const int v = q == 0 ? a[0] : q == 1 ? a[1] : q == 2 ? a[2] : a[3];
        return __builtin_amdgcn_readlane(v, l);
    };
    // one step: least key among this lane's nodes with stock and capacity, then the wave's
    auto step = [&](int jj, uint2 kc, uint2 bi) {
        const int s = lane_val(sv, jj);
        uint32_t xv = rows[s * WAVE + lane];
        const int a = cap_choose<POL>(kc, bi, (xv & 0xffu) && c0 > 0, (xv >> 8) && c1 > 0, c0,
                                      c1, lane, L.N - 1, L.gnum, L.gden, L.glow);
        if (a >= 0 && (a >> 1) == lane) {
            if (a & 1) { --c1; xv -= 0x100u; }
            else { --c0; xv -= 1u; }
            rows[s * WAVE + lane] = (uint16_t)xv;
        }
        if (lane == 0) out[jj] = a;
    };
    auto keys_at = [&](int jj) {
        return K2[(int64_t)lane_val(rg, jj < n ? jj : n - 1) * WAVE + lane];
    };
    auto bids_at = [&](int jj) {
        if constexpr (POL == CAP_BID) return bid_row(L, lane_val(sk, jj < n ? jj : n - 1), lane);
        else return make_uint2(0u, 0u);
    };
    uint2 k0 = keys_at(0), k1 = keys_at(1), k2 = keys_at(2), k3 = keys_at(3);
    uint2 b0 = bids_at(0), b1 = bids_at(1), b2 = bids_at(2), b3 = bids_at(3);
    for (int j = 0; j < n; j += 4) {
        step(j, k0, b0);
        k0 = keys_at(j + 4);
        b0 = bids_at(j + 4);
        if (j + 1 < n) step(j + 1, k1, b1);
        k1 = keys_at(j + 5);
        b1 = bids_at(j + 5);
        if (j + 2 < n) step(j + 2, k2, b2);
        k2 = keys_at(j + 6);
        b2 = bids_at(j + 6);
        if (j + 3 < n) step(j + 3, k3, b3);
        k3 = keys_at(j + 7);
        b3 = bids_at(j + 7);
    }
    __syncthreads();
    int nch = 0;
    const int pass = ctl->pass;
    for (int j = lane; j < n; j += WAVE) {
        const int a = out[j];
        if (a != L.alpha[lo + j]) {
            ++nch;
            L.skuchg[L.sku[lo + j]] = pass;
        }
        L.alpha[lo + j] = a;
    }
    nch = wave_sum(nch);
    if (lane == 0 && nch > 0) {
        atomicAdd(&L.chg[(pass - 1) % CAP_GROUP], nch);
        atomicMin(&ctl->first_blk, m);
    }
}

// Starts a pass: its number, its restart point (the previous pass's first changed block;
// INT_MAX after a pass without change, which makes the pass a no-op) and its change count
// (slot (pass - 1) % CAP_GROUP of chg: the host reads a group of passes at once).
__global__ void k_cap_pass_reset(CapPlan L, int first)
{
    if (threadIdx.x == 0) {
        CapCtl *ctl = L.ctl;
        const int pass = first ? 1 : ctl->pass + 1;
        ctl->pass = pass;
        ctl->frontier = first ? -1 : ctl->first_blk;
        ctl->first_blk = INT_MAX;
        L.chg[(pass - 1) % CAP_GROUP] = 0;
    }
}

__global__ void k_cap_fill(int32_t *p, int64_t n, int32_t v)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// Final stock and capacity from the converged actions (unit demand: every action ships
// one unit).
__global__ __launch_bounds__(256) void k_cap_final(CapPlan L, int32_t *final_inv, int32_t *used)
{
    __shared__ int32_t hist[CAP_NPAD];
    if (threadIdx.x < CAP_NPAD) hist[threadIdx.x] = 0;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < L.T; t += stride) {
        const int a = L.alpha[t];
        if (a >= 0) {
            atomicAdd(&hist[a], 1);
            if (final_inv) atomicSub(&final_inv[(int64_t)L.sku[t] * L.N + a], 1);
        }
    }
    __syncthreads();
    if (threadIdx.x < L.N && hist[threadIdx.x]) atomicAdd(&used[threadIdx.x], hist[threadIdx.x]);
}

// Final stock rows after convergence (every action of the fixed point ships one unit):
// the last piece of each SKU writes x0 minus the SKU's actions per node, counted from its
// piece prefix and its own positions (one ballot per distinct node per 64 positions).
// Rows of SKUs without orders keep the copy of x0 made before.
__global__ __launch_bounds__(256) void k_cap_final_rows(CapPlan L, int32_t *final_inv)
{
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int n_pieces = L.ctl->n_pieces, N = L.N;
    for (int p = uni(blockIdx.x * 4 + wave); p < n_pieces; p += gridDim.x * 4) {
        const int4 pd = L.piece[p]; // SKU, lo, hi, several pieces
        const int k = pd.x;
        if (p != L.piece_off[k + 1] - 1) continue; // not the SKU's last piece
        int ca = 0, cb = 0;
        if (pd.w) {
            const int32_t *row = L.pc + (int64_t)p * CAP_NPAD;
            ca = row[lane];
            cb = row[WAVE + lane];
        }
        for (int base = pd.y; base < pd.z; base += WAVE) {
            const int i = base + lane;
            const int a = i < pd.z ? L.alpha[L.perm[i]] : LOST;
            uint64_t rem = __ballot(a >= 0);
            while (rem) {
                const int q = __ffsll((long long)rem) - 1;
                const int v = uni(__shfl(a, q, WAVE));
                const uint64_t mv = __ballot(a == v);
                if (lane == (v & (WAVE - 1))) {
                    if (v < WAVE) ca += __popcll(mv);
                    else cb += __popcll(mv);
                }
                rem &= ~mv;
            }
        }
        int32_t *fr = final_inv + (int64_t)k * N;
        if (lane < N) fr[lane] = L.x0[(int64_t)k * N + lane] - ca;
        if (WAVE + lane < N) fr[WAVE + lane] = L.x0[(int64_t)k * N + WAVE + lane] - cb;
    }
}

__global__ void k_cap_final_cap(const int32_t *cap0, const int32_t *used, int N, int32_t *out)
{
    const int w = threadIdx.x;
    if (w < N) out[w] = cap0[w] - used[w];
}

// The serial sweep with capacity (the comparator): one wave, one order at a time in time
// order; stock rows in global memory (`state`, a copy of x0), capacities in registers.
// The next order's stock row and keys are loaded while the current order is decided; if
// both orders share the SKU, the loaded row is corrected by the current order's unit.
template <int POL>
__global__ __launch_bounds__(64) void k_cap_serial(CapPlan L, int32_t *state, int32_t *actions)
{
    const int lane = threadIdx.x, N = L.N;
    const int w0 = 2 * lane, w1 = 2 * lane + 1;
    int c0 = w0 < N ? L.cap0[w0] : 0, c1 = w1 < N ? L.cap0[w1] : 0;
    const uint2 *K2 = (const uint2 *)L.keyT;
    const int T = L.T;
    if (T == 0) return;
    // order data 64 at a time, one chunk ahead
    int csk = L.sku[min(lane, T - 1)], crg = L.region[min(lane, T - 1)];
    int nsk = L.sku[min(WAVE + lane, T - 1)], nrg = L.region[min(WAVE + lane, T - 1)];
    int k = uni(__shfl(csk, 0, WAVE)), r = uni(__shfl(crg, 0, WAVE));
    int xa = w0 < N ? state[(int64_t)k * N + w0] : 0, xb = w1 < N ? state[(int64_t)k * N + w1] : 0;
    uint2 kc = K2[(int64_t)r * WAVE + lane];
    uint2 bi = make_uint2(0u, 0u);
    if constexpr (POL == CAP_BID) bi = bid_row(L, k, lane);
    int abuf = LOST;
    for (int t = 0; t < T; ++t) {
        const int tn = t + 1;
        if ((tn & (WAVE - 1)) == 0 && tn < T) { // next chunk becomes current
            csk = nsk;
            crg = nrg;
            const int pf = min(tn + WAVE + lane, T - 1);
            nsk = L.sku[pf];
            nrg = L.region[pf];
        }
        int kn = k, rn = r;
        int xna = 0, xnb = 0;
        uint2 kn2 = kc, bn = bi;
        if (tn < T) {
            kn = uni(__shfl(csk, tn & (WAVE - 1), WAVE));
            rn = uni(__shfl(crg, tn & (WAVE - 1), WAVE));
            xna = w0 < N ? state[(int64_t)kn * N + w0] : 0;
            xnb = w1 < N ? state[(int64_t)kn * N + w1] : 0;
            kn2 = K2[(int64_t)rn * WAVE + lane];
            if constexpr (POL == CAP_BID) bn = bid_row(L, kn, lane);
        }
        const int a = cap_choose<POL>(kc, bi, xa > 0 && c0 > 0, xb > 0 && c1 > 0, c0, c1, lane,
                                      N - 1, L.gnum, L.gden, L.glow);
        if (a >= 0 && (a >> 1) == lane) {
            if (a & 1) {
                --c1;
                state[(int64_t)k * N + w1] = --xb;
                if (kn == k) --xnb;
            } else {
                --c0;
                state[(int64_t)k * N + w0] = --xa;
                if (kn == k) --xna;
            }
        }
        if (lane == (t & (WAVE - 1))) abuf = a;
        if ((t & (WAVE - 1)) == WAVE - 1 || t == T - 1) {
            const int base = t & ~(WAVE - 1);
            if (base + lane <= t) actions[base + lane] = abuf;
        }
        k = kn;
        r = rn;
        xa = xna;
        xb = xnb;
        kc = kn2;
        bi = bn;
    }
}

inline unsigned grid_for(int64_t n, int threads, int cap = 65535)
{
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

} // namespace

size_t cap_walk_lds(int B, int D) { return (size_t)D * CAP_NPAD + (size_t)(D + B) * 4; }

// Input checks of a capacity run (every later kernel indexes with these values): clears
// the control block and sets CapCtl::error.  init: the initial cache, nullable.
hipError_t cap_check(CapPlan &L, const int32_t *init, hipStream_t st)
{
    hipLaunchKernelGGL(k_cap_fill, dim3(1), dim3(64), 0, st, (int32_t *)L.ctl,
                       (int64_t)(sizeof(CapCtl) / 4), 0);
    hipLaunchKernelGGL(k_cap_check, dim3(grid_for(std::max<int64_t>(L.T, (int64_t)L.K * L.N), 256, 4096)),
                       dim3(256), 0, st, L, (int64_t)L.K * L.N, init);
    return hipGetLastError();
}

// Setup of a capacity run after cap_check passed: SKU sort, block slots and row ids,
// pieces, key table.  keys/vals/alt buffers and first hold T entries, tmp the larger of
// the radix-sort and scan scratch.
hipError_t cap_setup(CapPlan &L, int32_t *keys, int32_t *vals, int32_t *keys_alt,
                     int32_t *vals_alt, int32_t *first, void *tmp, hipStream_t st)
{
    hipError_t e;
    if (L.T == 0)
        hipLaunchKernelGGL(k_cap_fill, dim3(grid_for(L.K + 1, 256)), dim3(256), 0, st, L.seg_off,
                           (int64_t)L.K + 1, 0);
    hipLaunchKernelGGL(k_cap_keytab, dim3(grid_for((int64_t)L.R * CAP_NPAD, 256)), dim3(256), 0, st, L);
    if (L.T > 0) {
        hipLaunchKernelGGL(k_cap_keys, dim3(grid_for(L.T, 256, 8192)), dim3(256), 0, st, L, keys,
                           vals);
        int bits = 1;
        while (bits < 31 && (1ll << bits) < L.K) ++bits;
        bool in_alt = false;
        if ((e = radix_sort_pairs(keys, vals, keys_alt, vals_alt, L.T, bits, tmp, st, &in_alt)) !=
            hipSuccess)
            return e;
        const int32_t *sorted = in_alt ? vals_alt : vals;
        hipLaunchKernelGGL(k_cap_seg_bounds, dim3(grid_for(L.T + 1, 256, 8192)), dim3(256), 0, st,
                           L, in_alt ? keys_alt : keys);
        if ((e = hipMemcpyAsync(L.perm, sorted, (size_t)L.T * 4, hipMemcpyDeviceToDevice, st)) !=
            hipSuccess)
            return e;
        hipLaunchKernelGGL(k_cap_slots, dim3(L.nblk), dim3(64), 0, st, L, first);
        if ((e = hipMemcpyAsync(L.sid, first, (size_t)L.T * 4, hipMemcpyDeviceToDevice, st)) !=
            hipSuccess)
            return e;
        if ((e = scan_i32_excl(L.sid, L.T, tmp, st)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_cap_srow, dim3(grid_for(L.T, 256, 8192)), dim3(256), 0, st, L);
    }
    hipLaunchKernelGGL(k_cap_piece_counts, dim3(grid_for((int64_t)L.K + 1, 256)), dim3(256), 0, st, L,
                       L.piece_off);
    if ((e = scan_i32_excl(L.piece_off, (int64_t)L.K + 1, tmp, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_cap_piece_fill, dim3(grid_for(L.K, 256)), dim3(256), 0, st, L);
    return hipGetLastError();
}

// One Picard pass (launches only; the caller reads ctl afterwards).
hipError_t cap_pass(const CapPlan &L, bool first, hipStream_t st)
{
    hipLaunchKernelGGL(k_cap_pass_reset, dim3(1), dim3(64), 0, st, L, first ? 1 : 0);
    if (L.T == 0) return hipGetLastError();
    // grid-stride launches: about eight 4-wave workgroups per CU loop over the pieces
    // (most pieces are a rare SKU's few orders; one workgroup each would make the launch
    // bound by workgroup dispatch)
    const unsigned cap_wg = 8 * 256;
    const unsigned gp = (unsigned)std::min<int64_t>((L.max_pieces + 3) / 4, cap_wg);
    const unsigned gk = (unsigned)std::min<int64_t>(L.K, cap_wg);
    hipLaunchKernelGGL(k_cap_piece_count, dim3(gp), dim3(256), 0, st, L);
    hipLaunchKernelGGL(k_cap_piece_scan, dim3(gk), dim3(256), 0, st, L);
    hipLaunchKernelGGL(k_cap_entry, dim3(gp), dim3(256), 0, st, L);
    hipLaunchKernelGGL(k_cap_hist, dim3((unsigned)((L.nblk + 3) / 4)), dim3(256), 0, st, L);
    hipLaunchKernelGGL(k_cap_scan, dim3(L.N), dim3(CAP_SCAN_T), 0, st, L);
    const size_t lds = cap_walk_lds(L.B, L.dmax);
    if (L.pol == CAP_GREEDY)
        hipLaunchKernelGGL(k_cap_walk<CAP_GREEDY>, dim3(L.nblk), dim3(64), lds, st, L);
    else if (L.pol == CAP_GAMMA)
        hipLaunchKernelGGL(k_cap_walk<CAP_GAMMA>, dim3(L.nblk), dim3(64), lds, st, L);
    else
        hipLaunchKernelGGL(k_cap_walk<CAP_BID>, dim3(L.nblk), dim3(64), lds, st, L);
    return hipGetLastError();
}

hipError_t cap_finish(const CapPlan &L, int32_t *final_inv, int32_t *final_cap, int32_t *used,
                      hipStream_t st)
{
    hipError_t e;
    hipLaunchKernelGGL(k_cap_fill, dim3(1), dim3(128), 0, st, used, (int64_t)L.N, 0);
    if (final_inv) {
        if ((e = hipMemcpyAsync(final_inv, L.x0, (size_t)L.K * L.N * 4, hipMemcpyDeviceToDevice,
                                st)) != hipSuccess)
            return e;
        if (L.T > 0)
            hipLaunchKernelGGL(k_cap_final_rows,
                               dim3((unsigned)std::min<int64_t>((L.max_pieces + 3) / 4, 8 * 256)),
                               dim3(256), 0, st, L, final_inv);
    }
    hipLaunchKernelGGL(k_cap_final, dim3(grid_for(L.T, 256, 2048)), dim3(256), 0, st, L, nullptr,
                       used);
    if (final_cap)
        hipLaunchKernelGGL(k_cap_final_cap, dim3(1), dim3(CAP_NPAD), 0, st, L.cap0, used, L.N,
                           final_cap);
    return hipGetLastError();
}

hipError_t cap_serial_setup(CapPlan &L, hipStream_t st)
{
    hipLaunchKernelGGL(k_cap_keytab, dim3(grid_for((int64_t)L.R * CAP_NPAD, 256)), dim3(256), 0, st, L);
    return hipGetLastError();
}

hipError_t cap_serial(const CapPlan &L, int32_t *state, int32_t *actions, hipStream_t st)
{
    if (L.pol == CAP_GREEDY)
        hipLaunchKernelGGL(k_cap_serial<CAP_GREEDY>, dim3(1), dim3(64), 0, st, L, state, actions);
    else if (L.pol == CAP_GAMMA)
        hipLaunchKernelGGL(k_cap_serial<CAP_GAMMA>, dim3(1), dim3(64), 0, st, L, state, actions);
    else
        hipLaunchKernelGGL(k_cap_serial<CAP_BID>, dim3(1), dim3(64), 0, st, L, state, actions);
    return hipGetLastError();
}

} // namespace pk

// Picard iteration with node capacity (Section 3: the FO state is (x_t, c_t); an order of
// SKU i may go to node j only while c_{t,j} > 0 and x_{t,i,j} > 0; shipping one unit lowers
// both).  Unit demand, greedy policy (least cost, lowest index on ties), one trajectory.
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
//  2. k_cap_entry: one wave per piece walks its positions of the SKU-sorted list; at
//     the first order of each (block, SKU) it writes that block's stock row of the SKU
//     (clamped to 255: a block walk takes at most B <= 255 units from it), and it adds
//     each (block, SKU)'s passing actions to the block's node counts H;
//  3. k_cap_scan: per node, exclusive scan of H over blocks -> entry capacities;
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

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v)
{
    for (int d = WAVE / 2; d > 0; d >>= 1) {
        const uint32_t o = (uint32_t)__shfl_xor((int)v, d, WAVE);
        v = o < v ? o : v;
    }
    return v;
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
    if (err) atomicOr(&L.ctl->error, err);
}

__global__ void k_cap_keys(CapPlan L, int32_t *keys, int32_t *vals, int32_t *hist)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < L.T; t += stride) {
        const int32_t k = L.sku[t];
        keys[t] = k;
        vals[t] = (int32_t)t;
        atomicAdd(&hist[k], 1);
    }
}

// Greedy keys, region-major: one 512-byte row per region.
__global__ void k_cap_keytab(CapPlan L)
{
    const int64_t n = (int64_t)L.R * CAP_NPAD;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int r = (int)(i / CAP_NPAD), w = (int)(i % CAP_NPAD);
        L.keyT[i] = w < L.N ? ((uint32_t)L.cost[(int64_t)w * L.R + r] << 8) | (uint32_t)w : CAP_NONE;
    }
}

// One wave per block: the index in the block of the first order of each order's SKU, and
// a 0/1 flag for first orders (scanned into row ids afterwards).
__global__ __launch_bounds__(64) void k_cap_slots(CapPlan L, int32_t *first)
{
    __shared__ int32_t sk[CAP_MAX_B];
    const int m = blockIdx.x, lane = threadIdx.x;
    const int lo = m * L.B, hi = min(lo + L.B, L.T), n = hi - lo;
    for (int j = lane; j < n; j += WAVE) sk[j] = L.sku[lo + j];
    __syncthreads();
    for (int j = lane; j < n; j += WAVE) {
        int f = j;
        for (int i = 0; i < j; ++i)
            if (sk[i] == sk[j]) { f = i; break; }
        L.slot[lo + j] = f;
        first[lo + j] = f == j;
    }
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

__global__ void k_cap_piece_fill(CapPlan L)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < L.K; k += stride) {
        for (int p = L.piece_off[k]; p < L.piece_off[k + 1]; ++p) L.piece_seg[p] = (int32_t)k;
        if (k == L.K - 1) L.ctl->n_pieces = L.piece_off[L.K];
    }
}

// ---------------------------------------------------------------- one pass
// Piece p of SKU k covers sorted positions [seg_off[k] + j*CAP_PIECE, ...) with j its
// index in the SKU.
__device__ __forceinline__ void piece_range(const CapPlan &L, int p, int &k, int &j, int &lo,
                                            int &hi)
{
    k = L.piece_seg[p];
    j = p - L.piece_off[k];
    lo = L.seg_off[k] + j * CAP_PIECE;
    hi = min(lo + CAP_PIECE, L.seg_off[k + 1]);
}

// Cached action counts per piece of the SKUs with more than one piece.
__global__ __launch_bounds__(256) void k_cap_piece_count(CapPlan L)
{
    __shared__ int32_t u[4][CAP_NPAD];
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int p = uni(blockIdx.x * 4 + wave);
    if (p >= L.ctl->n_pieces) return;
    int k, j, lo, hi;
    piece_range(L, p, k, j, lo, hi);
    if (L.piece_off[k + 1] - L.piece_off[k] < 2) return;
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
}

// Exclusive scan of the piece counts along each SKU with more than one piece.
__global__ __launch_bounds__(256) void k_cap_piece_scan(CapPlan L)
{
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int k = uni(blockIdx.x * 4 + wave);
    if (k >= L.K) return;
    const int p0 = L.piece_off[k], p1 = L.piece_off[k + 1];
    if (p1 - p0 < 2) return;
    int run0 = 0, run1 = 0;
    for (int p = p0; p < p1; ++p) {
        int32_t *row = L.pc + (int64_t)p * CAP_NPAD;
        const int v0 = row[lane], v1 = row[WAVE + lane];
        row[lane] = run0;
        row[WAVE + lane] = run1;
        run0 += v0;
        run1 += v1;
    }
}

// One wave per piece: stock rows at each (block, SKU)'s first order and passing cached
// actions per (node, block).  Lane l holds nodes l and 64 + l.
__global__ __launch_bounds__(256) void k_cap_entry(CapPlan L)
{
    __shared__ int32_t ush[4][CAP_NPAD];
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int p = uni(blockIdx.x * 4 + wave);
    if (p >= L.ctl->n_pieces) return;
    int k, j, lo, hi;
    piece_range(L, p, k, j, lo, hi);
    int32_t *u = ush[wave];
    const int N = L.N, B = L.B, nblk = L.nblk;
    const int frontier = L.ctl->frontier;
    const int w0 = lane, w1 = WAVE + lane;
    const int x0a = w0 < N ? L.x0[(int64_t)k * N + w0] : 0;
    const int x0b = w1 < N ? L.x0[(int64_t)k * N + w1] : 0;
    int ca = 0, cb = 0; // cached actions of this SKU to each node before the position
    if (L.piece_off[k + 1] - L.piece_off[k] > 1) {
        const int32_t *row = L.pc + (int64_t)p * CAP_NPAD;
        ca = row[w0];
        cb = row[w1];
    }
    u[w0] = 0;
    u[w1] = 0;
    wave_sync();
    int cur = -1; // block of the (block, SKU) being accumulated
    auto flush = [&](int m) {
        wave_sync();
        const int ua = u[w0], ub = u[w1];
        const int pa = min(ua, max(0, x0a - ca)), pb = min(ub, max(0, x0b - cb));
        if (pa > 0) atomicAdd(&L.H[(int64_t)w0 * nblk + m], pa);
        if (pb > 0) atomicAdd(&L.H[(int64_t)w1 * nblk + m], pb);
        ca += ua;
        cb += ub;
        u[w0] = 0;
        u[w1] = 0;
        wave_sync();
    };
    for (int base = lo; base < hi; base += WAVE) {
        const int i = base + lane;
        const bool valid = i < hi;
        const int t = valid ? L.perm[i] : 0;
        const int m = valid ? t / B : INT_MAX;
        const int a = valid ? L.alpha[t] : LOST;
        const bool first = valid && L.slot[t] == t - m * B;
        const uint64_t vmask = __ballot(valid);
        uint64_t done = 0;
        while (done != vmask) { // pieces of equal block, in lane order
            const int p0 = __ffsll((long long)(vmask & ~done)) - 1;
            const int mm = uni(__shfl(m, p0, WAVE));
            if (mm != cur) {
                if (cur >= 0) flush(cur);
                cur = mm;
                const int f = __shfl((int)first, p0, WAVE);
                if (f && mm > frontier) { // the block's stock row of this SKU
                    const int tp = __shfl(t, p0, WAVE);
                    uint8_t *xr = L.X + (int64_t)L.sid[tp] * CAP_NPAD;
                    xr[w0] = clamp255(x0a - ca);
                    xr[w1] = clamp255(x0b - cb);
                }
            }
            const bool in = valid && m == mm;
            if (in && a >= 0) atomicAdd(&u[a], 1);
            done |= __ballot(in);
        }
    }
    if (cur >= 0) flush(cur);
}

// Per node, exclusive scan of the passing counts over blocks: capacity at each block's
// start.  Clears H for the next pass.
__global__ __launch_bounds__(256) void k_cap_scan(CapPlan L)
{
    __shared__ int32_t part[256];
    const int w = blockIdx.x, tid = threadIdx.x;
    const int nblk = L.nblk;
    const int per = (nblk + 255) / 256;
    const int b0 = tid * per, b1 = min(b0 + per, nblk);
    int32_t *h = L.H + (int64_t)w * nblk;
    int s = 0;
    for (int b = b0; b < b1; ++b) s += h[b];
    part[tid] = s;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
        const int v = tid >= d ? part[tid - d] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int run = tid > 0 ? part[tid - 1] : 0;
    const int c0 = L.cap0[w];
    for (int b = b0; b < b1; ++b) {
        const int v = h[b];
        h[b] = 0;
        L.capE[(int64_t)b * CAP_NPAD + w] = max(0, c0 - run);
        run += v;
    }
}

// One wave per block: the block's orders in time order with fresh greedy decisions.
// Lane l holds nodes 2l and 2l+1 (stock bytes as one 16-bit LDS word, capacities and keys
// in registers).  A lane writes only its own stock word, so steps need no barrier.
__global__ __launch_bounds__(64) void k_cap_walk(CapPlan L)
{
    extern __shared__ __align__(16) unsigned char cap_smem[];
    const int m = blockIdx.x, lane = threadIdx.x;
    CapCtl *ctl = L.ctl;
    if (m <= ctl->frontier) return;
    const int B = L.B;
    const int lo = m * B, hi = min(lo + B, L.T), n = hi - lo;
    uint16_t *rows = (uint16_t *)cap_smem;              // [B][64] stock words
    int32_t *reg = (int32_t *)(cap_smem + (size_t)B * CAP_NPAD); // [B]
    int32_t *sl = reg + B;                                // [B]
    int32_t *out = sl + B;                                // [B]
    for (int j = lane; j < n; j += WAVE) {
        reg[j] = L.region[lo + j];
        sl[j] = L.slot[lo + j];
    }
    __syncthreads();
    const uint16_t *X16 = (const uint16_t *)L.X;
    for (int j = 0; j < n; ++j)
        if (sl[j] == j) rows[j * WAVE + lane] = X16[(int64_t)L.sid[lo + j] * WAVE + lane];
    const int2 cv = *(const int2 *)(L.capE + (int64_t)m * CAP_NPAD + 2 * lane);
    int c0 = 2 * lane < L.N ? cv.x : 0, c1 = 2 * lane + 1 < L.N ? cv.y : 0;
    const uint2 *K2 = (const uint2 *)L.keyT;
    uint2 kc = K2[(int64_t)reg[0] * WAVE + lane];
    for (int j = 0; j < n; ++j) {
        const int jn = j + 1 < n ? j + 1 : j;
        const uint2 kn = K2[(int64_t)reg[jn] * WAVE + lane]; // next step's keys
        const int s = sl[j];
        uint32_t xv = rows[s * WAVE + lane];
        const uint32_t ka = ((xv & 0xffu) && c0 > 0) ? kc.x : CAP_NONE;
        const uint32_t kb = ((xv >> 8) && c1 > 0) ? kc.y : CAP_NONE;
        const uint32_t best = wave_min_u32(ka < kb ? ka : kb);
        const int a = best == CAP_NONE ? LOST : (int)(best & 0xffu);
        if (a >= 0 && (a >> 1) == lane) {
            if (a & 1) { --c1; xv -= 0x100u; }
            else { --c0; xv -= 1u; }
            rows[s * WAVE + lane] = (uint16_t)xv;
        }
        if (lane == 0) out[j] = a;
        kc = kn;
    }
    __syncthreads();
    int nch = 0;
    for (int j = lane; j < n; j += WAVE) {
        const int a = out[j];
        nch += a != L.alpha[lo + j];
        L.alpha[lo + j] = a;
    }
    nch = wave_sum(nch);
    if (lane == 0 && nch > 0) {
        atomicAdd(&ctl->changed, nch);
        atomicMin(&ctl->first_blk, m);
    }
}

__global__ void k_cap_pass_reset(CapCtl *ctl, int first)
{
    if (threadIdx.x == 0) {
        ctl->frontier = first ? -1 : (ctl->first_blk == INT_MAX ? INT_MAX : ctl->first_blk);
        ctl->changed = 0;
        ctl->first_blk = INT_MAX;
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

__global__ void k_cap_final_cap(const int32_t *cap0, const int32_t *used, int N, int32_t *out)
{
    const int w = threadIdx.x;
    if (w < N) out[w] = cap0[w] - used[w];
}

// The serial sweep with capacity (the comparator): one wave, one order at a time in time
// order; stock rows in global memory (`state`, a copy of x0), capacities in registers.
// The next order's stock row and keys are loaded while the current order is decided; if
// both orders share the SKU, the loaded row is corrected by the current order's unit.
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
        uint2 kn2 = kc;
        if (tn < T) {
            kn = uni(__shfl(csk, tn & (WAVE - 1), WAVE));
            rn = uni(__shfl(crg, tn & (WAVE - 1), WAVE));
            xna = w0 < N ? state[(int64_t)kn * N + w0] : 0;
            xnb = w1 < N ? state[(int64_t)kn * N + w1] : 0;
            kn2 = K2[(int64_t)rn * WAVE + lane];
        }
        const uint32_t ka = (xa > 0 && c0 > 0) ? kc.x : CAP_NONE;
        const uint32_t kb = (xb > 0 && c1 > 0) ? kc.y : CAP_NONE;
        const uint32_t best = wave_min_u32(ka < kb ? ka : kb);
        const int a = best == CAP_NONE ? LOST : (int)(best & 0xffu);
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

size_t cap_walk_lds(int B) { return (size_t)B * CAP_NPAD + (size_t)3 * B * 4; }

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
    hipLaunchKernelGGL(k_cap_fill, dim3(grid_for(L.K + 1, 256)), dim3(256), 0, st, L.seg_off,
                       (int64_t)L.K + 1, 0);
    hipLaunchKernelGGL(k_cap_keytab, dim3(grid_for((int64_t)L.R * CAP_NPAD, 256)), dim3(256), 0, st, L);
    if (L.T > 0) {
        hipLaunchKernelGGL(k_cap_keys, dim3(grid_for(L.T, 256, 8192)), dim3(256), 0, st, L, keys,
                           vals, L.seg_off);
        if ((e = scan_i32_excl(L.seg_off, (int64_t)L.K + 1, tmp, st)) != hipSuccess) return e;
        int bits = 1;
        while (bits < 31 && (1ll << bits) < L.K) ++bits;
        bool in_alt = false;
        if ((e = radix_sort_pairs(keys, vals, keys_alt, vals_alt, L.T, bits, tmp, st, &in_alt)) !=
            hipSuccess)
            return e;
        const int32_t *sorted = in_alt ? vals_alt : vals;
        if ((e = hipMemcpyAsync(L.perm, sorted, (size_t)L.T * 4, hipMemcpyDeviceToDevice, st)) !=
            hipSuccess)
            return e;
        hipLaunchKernelGGL(k_cap_slots, dim3(L.nblk), dim3(64), 0, st, L, first);
        if ((e = hipMemcpyAsync(L.sid, first, (size_t)L.T * 4, hipMemcpyDeviceToDevice, st)) !=
            hipSuccess)
            return e;
        if ((e = scan_i32_excl(L.sid, L.T, tmp, st)) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_cap_piece_counts, dim3(grid_for((int64_t)L.K + 1, 256)), dim3(256), 0, st, L,
                       L.piece_off);
    if ((e = scan_i32_excl(L.piece_off, (int64_t)L.K + 1, tmp, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_cap_piece_fill, dim3(grid_for(L.K, 256)), dim3(256), 0, st, L);
    hipLaunchKernelGGL(k_cap_fill, dim3(grid_for((int64_t)L.N * L.nblk, 256, 8192)), dim3(256), 0,
                       st, L.H, (int64_t)L.N * L.nblk, 0);
    return hipGetLastError();
}

// One Picard pass (launches only; the caller reads ctl afterwards).
hipError_t cap_pass(const CapPlan &L, bool first, hipStream_t st)
{
    hipLaunchKernelGGL(k_cap_pass_reset, dim3(1), dim3(64), 0, st, L.ctl, first ? 1 : 0);
    if (L.T == 0) return hipGetLastError();
    const unsigned gp = (unsigned)((L.max_pieces + 3) / 4);
    hipLaunchKernelGGL(k_cap_piece_count, dim3(gp), dim3(256), 0, st, L);
    hipLaunchKernelGGL(k_cap_piece_scan, dim3((unsigned)((L.K + 3) / 4)), dim3(256), 0, st, L);
    hipLaunchKernelGGL(k_cap_entry, dim3(gp), dim3(256), 0, st, L);
    hipLaunchKernelGGL(k_cap_scan, dim3(L.N), dim3(256), 0, st, L);
    hipLaunchKernelGGL(k_cap_walk, dim3(L.nblk), dim3(64), cap_walk_lds(L.B), st, L);
    return hipGetLastError();
}

hipError_t cap_finish(const CapPlan &L, int32_t *final_inv, int32_t *final_cap, int32_t *used,
                      hipStream_t st)
{
    hipError_t e;
    hipLaunchKernelGGL(k_cap_fill, dim3(1), dim3(128), 0, st, used, (int64_t)L.N, 0);
    if (final_inv &&
        (e = hipMemcpyAsync(final_inv, L.x0, (size_t)L.K * L.N * 4, hipMemcpyDeviceToDevice, st)) !=
            hipSuccess)
        return e;
    hipLaunchKernelGGL(k_cap_final, dim3(grid_for(L.T, 256, 2048)), dim3(256), 0, st, L, final_inv,
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
    hipLaunchKernelGGL(k_cap_serial, dim3(1), dim3(64), 0, st, L, state, actions);
    return hipGetLastError();
}

} // namespace pk

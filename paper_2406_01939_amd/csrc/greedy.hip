// The serial sweep under the greedy policy (Section 3.1, inventory as the constraint):
// among warehouses with stock, the least cost[w][region], lowest index on ties; lost
// sale iff none has stock.  With pos[b][r][w] the position of w in region r's
// (cost, index) order, the choice is the warehouse with stock of least position.  The
// sweep reads key[b][r][w] = (pos << S) | w (16-bit keys with S = 8 when N <= 256, else
// 32-bit keys with S = 16): the least key among warehouses with stock names the choice.
#include "greedy_keys.h"

namespace pk {

namespace {

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

// Minimum of an unsigned value over the 64 lanes of the wave (DPP: row shifts, then the
// row broadcasts; the result is read from lane 63).
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v)
{
#define PK_MIN_DPP(ctrl, rmask)                                                                  \
    {                                                                                            \
        const uint32_t o = (uint32_t)__builtin_amdgcn_update_dpp((int)0xffffffffu, (int)v, ctrl, \
                                                                 rmask, 0xf, false);             \
        v = o < v ? o : v;                                                                       \
    }
    PK_MIN_DPP(0x111, 0xf) // row_shr:1
    PK_MIN_DPP(0x112, 0xf) // row_shr:2
    PK_MIN_DPP(0x114, 0xf) // row_shr:4
    PK_MIN_DPP(0x118, 0xf) // row_shr:8
    PK_MIN_DPP(0x142, 0xa) // row_bcast:15 into rows 1 and 3
    PK_MIN_DPP(0x143, 0xc) // row_bcast:31 into rows 2 and 3
#undef PK_MIN_DPP
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Latency-bound serial sweep for N <= 128 (16-bit keys, two warehouses per lane: w = lane
// and lane + 64).  One wave per trajectory, one order at a time, with nothing but LDS and
// registers on an order's dependent path:
//  * the trajectory's key table sits in LDS;
//  * the orders' (SKU, region, quantity) are read 64 at a time into registers, the next 64
//    a chunk ahead; actions and units shipped leave 64 at a time;
//  * the stock row of order i + DIST is loaded into registers while order i is decided
//    (a ring of RING row slots), so its memory latency overlaps DIST orders;
//  * a row loaded before an order of the same SKU in between was decided is stale: the
//    order takes the row of the most recent such order (still in its slot) instead;
//  * the lane that holds warehouse a's stock also stores it back, so the load of a later
//    prefetch, by the same lane, sees the store (program order of one work-item).
constexpr int SER_DIST = 8;
constexpr int SER_RING = 16; // DIST slots ahead, DIST - 1 behind for the same-SKU check

__device__ __forceinline__ void ser_order_at(const Prob &P, int64_t t, int64_t t1, int &k, int &r,
                                             int &q)
{
    if (t < t1) {
        k = P.sku[t];
        r = P.region[t];
        q = P.qty[t];
        k = k < 0 ? 0 : (k >= P.K ? P.K - 1 : k); // out-of-range input never indexes memory
        r = r < 0 ? 0 : (r >= P.R ? P.R - 1 : r);
        q = q < 1 ? 1 : q;
    } else {
        k = 0;
        r = 0;
        q = 1;
    }
}

__global__ __launch_bounds__(64) void k_serial_greedy_pipe(Prob P, const uint16_t *keys,
                                                           int32_t *state, int32_t *actions,
                                                           int32_t *shipped)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int b = blockIdx.x;
    if (b >= P.n_traj) return;
    const int lane = threadIdx.x;
    const int N = P.N, R = P.R;
    const int npad = tab_npad<uint16_t>(N);
    const int64_t t0 = P.traj_off[b], t1 = P.traj_off[b + 1];
    const int64_t T = t1 - t0;
    if (T <= 0) return;
    int32_t *xs = state + (int64_t)b * P.K * N;
    { // the trajectory's key table into LDS
        const uint4 *src = (const uint4 *)(keys + b * tab_stride<uint16_t>(N, R));
        uint4 *dst = (uint4 *)smem;
        const int n16 = (int)(tab_stride<uint16_t>(N, R) * 2 / 16);
        for (int i = lane; i < n16; i += WAVE) dst[i] = src[i];
    }
    const uint16_t *tab = (const uint16_t *)smem;
    const bool w0 = lane < N, w1 = lane + WAVE < N;
    // order chunks: c holds orders t0 + 64 c + lane
    int ck, cr, cq, nk, nr, nq;
    ser_order_at(P, t0 + lane, t1, ck, cr, cq);
    ser_order_at(P, t0 + WAVE + lane, t1, nk, nr, nq);
    int32_t xa[SER_RING], xb[SER_RING]; // stock of warehouses lane and lane + 64, per slot
    int sk[SER_RING];                   // SKU of the order in each slot (wave-uniform)
#pragma unroll
    for (int u = 0; u < SER_RING; ++u) {
        xa[u] = xb[u] = 0;
        sk[u] = -1;
    }
    // loads are issued unconditionally (addresses clamped into the row, values masked):
    // no branch around them, so the compiler can wait for each one exactly DIST orders
    // later instead of for every outstanding load
    const int l0 = w0 ? lane : 0, l1 = w1 ? lane + WAVE : 0;
#pragma unroll
    for (int u = 0; u < SER_DIST; ++u) { // rows of orders 0 .. DIST-1 (orders past T: row 0)
        const int k = __builtin_amdgcn_readlane(ck, u);
        const int32_t *row = xs + (int64_t)k * N;
        xa[u] = row[l0];
        xb[u] = row[l1];
    }
    __syncthreads(); // the key table
    int act = LOST, shp = 0; // this chunk's outputs, lane l: order 64 c + l
    for (int64_t g = 0; g < T; g += SER_RING) {
#pragma unroll
        for (int u = 0; u < SER_RING; ++u) {
            const int64_t i = g + u;
            if (i >= T) continue; // the last group's tail (wave-uniform)
            const int li = (int)(i & (WAVE - 1));
            if (li == 0 && i > 0) { // next chunk
                ck = nk;
                cr = nr;
                cq = nq;
                ser_order_at(P, t0 + i + WAVE + lane, t1, nk, nr, nq);
                act = LOST;
                shp = 0;
            }
            const int k = __builtin_amdgcn_readlane(ck, li);
            const int r = __builtin_amdgcn_readlane(cr, li);
            const int q = __builtin_amdgcn_readlane(cq, li);
            // the row: this slot's prefetch, unless an order of the same SKU was decided
            // after it was loaded (the most recent one's slot holds the current row)
            int32_t x0v = xa[u], x1v = xb[u];
#pragma unroll
            for (int j = SER_DIST - 1; j >= 1; --j) {
                const int v = (u - j) & (SER_RING - 1);
                if (i >= j && sk[v] == k) {
                    x0v = xa[v];
                    x1v = xb[v];
                }
            }
            sk[u] = k;
            const uint16_t *kr = tab + (int64_t)r * npad;
            const uint32_t k0 = w0 && x0v > 0 ? (uint32_t)kr[l0] : 0xffffffffu;
            const uint32_t k1 = w1 && x1v > 0 ? (uint32_t)kr[l1] : 0xffffffffu;
            const uint32_t best = wave_min_u32(k0 < k1 ? k0 : k1);
            int a = LOST, sh = 0;
            if (best != 0xffffffffu) {
                a = (int)(best & 0xffu);
                const int own = a & (WAVE - 1);
                const int32_t xv = __builtin_amdgcn_readlane(a < WAVE ? x0v : x1v, own);
                sh = q < xv ? q : xv;
                if (lane == own) {
                    if (a < WAVE) x0v -= sh;
                    else x1v -= sh;
                    xs[(int64_t)k * N + a] = xv - sh;
                }
            }
            xa[u] = x0v;
            xb[u] = x1v;
            if (lane == li) {
                act = a;
                shp = sh;
            }
            if (li == WAVE - 1 || i == T - 1) { // the chunk's outputs
                const int64_t to = t0 + (i - li) + lane;
                if (lane <= li) {
                    actions[to] = act;
                    if (shipped) shipped[to] = shp;
                }
            }
            // prefetch: the row of order i + DIST into slot (u + DIST) % RING (an order past
            // the end reads row 0: its slot is never used)
            const int lp = (int)((i + SER_DIST) & (WAVE - 1));
            const int kp = __builtin_amdgcn_readlane(lp > li ? ck : nk, lp);
            const int32_t *row = xs + (int64_t)kp * N;
            xa[(u + SER_DIST) & (SER_RING - 1)] = row[l0];
            xb[(u + SER_DIST) & (SER_RING - 1)] = row[l1];
        }
    }
}

// key[b][r][w] = (position of w in region r's increasing (cost[b][w][r], w) order) << S
// | w.  One workgroup per row (b, r): the row's costs are staged in LDS, then one thread
// per w counts the warehouses that precede it.  Row padding is all-ones.  With pref (16-bit
// keys, N <= 128) the row's preference list too: pref[b][r][position] = w.
template <typename KeyT>
__global__ __launch_bounds__(256) void k_keys(Prob P, KeyT *keys, uint8_t *pref)
{
    __shared__ int32_t cs[PK_MAX_WAREHOUSES];
    const int N = P.N, R = P.R;
    const int npad = tab_npad<KeyT>(N);
    const int64_t nrows = (int64_t)P.n_traj * R;
    for (int64_t br = blockIdx.x; br < nrows; br += gridDim.x) {
        const int r = (int)(br % R);
        const int64_t b = br / R;
        const int32_t *c = P.cost + b * N * R;
        __syncthreads(); // the previous row's counts are done with cs
        for (int v = threadIdx.x; v < N; v += blockDim.x) cs[v] = c[(int64_t)v * R + r];
        __syncthreads();
        KeyT *row = keys + b * tab_stride<KeyT>(N, R) + (int64_t)r * npad;
        uint8_t *prow = pref ? pref + br * pref_npad(N) : nullptr; // pref_npad(N) == npad here
        for (int w = threadIdx.x; w < npad; w += blockDim.x) {
            if (w >= N) {
                row[w] = (KeyT)~(KeyT)0;
                if (prow) prow[w] = 127; // positions past N
                continue;
            }
            const int32_t cw = cs[w];
            uint32_t q = 0;
            for (int v = 0; v < N; ++v) {
                const int32_t cv = cs[v];
                q += (cv < cw) || (cv == cw && v < w);
            }
            row[w] = (KeyT)((q << key_shift<KeyT>()) | (uint32_t)w);
            if (prow) prow[q] = (uint8_t)w;
        }
    }
}

} // namespace

bool keys16(int N) { return N <= 255; } // the all-ones key 0xffff is the no-stock sentinel

size_t pos_bytes(int N, int R, int n_traj)
{
    return keys16(N) ? (size_t)n_traj * tab_stride<uint16_t>(N, R) * 2
                     : (size_t)n_traj * tab_stride<uint32_t>(N, R) * 4;
}

size_t pref_bytes(int N, int R, int n_traj)
{
    return N <= PREF_MAX_N ? (size_t)n_traj * R * pref_npad(N) : 0;
}

hipError_t setup_pos(const Prob &P, void *keys, uint8_t *pref, hipStream_t st)
{
    int64_t g = (int64_t)P.n_traj * P.R; // one workgroup per row
    g = g < 1 ? 1 : (g > 8192 ? 8192 : g);
    const int threads = P.N <= 128 ? 128 : 256;
    if (keys16(P.N))
        hipLaunchKernelGGL(k_keys<uint16_t>, dim3((unsigned)g), dim3(threads), 0, st, P,
                           (uint16_t *)keys, P.N <= PREF_MAX_N ? pref : nullptr);
    else
        hipLaunchKernelGGL(k_keys<uint32_t>, dim3((unsigned)g), dim3(threads), 0, st, P,
                           (uint32_t *)keys, (uint8_t *)nullptr);
    return hipGetLastError();
}

hipError_t launch_serial_greedy(const Prob &P, const void *keys, int32_t *state, int32_t *actions,
                                int32_t *shipped, hipStream_t st)
{
    const size_t tab_b = (size_t)tab_stride<uint16_t>(P.N, P.R) * 2;
    if (P.N <= 2 * WAVE && tab_b <= 64 * 1024)
        hipLaunchKernelGGL(k_serial_greedy_pipe, dim3(P.n_traj), dim3(64), tab_b, st, P,
                           (const uint16_t *)keys, state, actions, shipped);
    else if (keys16(P.N))
        hipLaunchKernelGGL(k_serial_greedy<uint16_t>, dim3(P.n_traj), dim3(64), 0, st, P,
                           (const uint16_t *)keys, state, actions, shipped);
    else
        hipLaunchKernelGGL(k_serial_greedy<uint32_t>, dim3(P.n_traj), dim3(64), 0, st, P,
                           (const uint32_t *)keys, state, actions, shipped);
    return hipGetLastError();
}

} // namespace pk

// The serial sweep under the greedy policy (Section 3.1, inventory as the constraint):
// among warehouses with stock, the least cost[w][region], lowest index on ties; lost
// sale iff none has stock.  With pos[b][r][w] the position of w in region r's
// (cost, index) order, the choice is the warehouse with stock of least position.  The
// sweep reads key[b][r][w] = (pos << S) | w (16-bit keys with S = 8 when N <= 256, else
// 32-bit keys with S = 16): the least key among warehouses with stock names the choice.
#include <climits>
#include <type_traits>

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

// Latency-bound serial sweep for N <= 128 (two warehouses per lane: w = lane and
// lane + 64).  One wave per trajectory decides one order at a time; a wave issues one
// instruction per issue cycle of its SIMD, so the sweep's speed is the instruction count
// of an order's code plus the latencies that are not hidden.  Hence:
//  * the key table sits in LDS as pairs, one 32-bit word per lane and region (keys of
//    warehouses lane and lane + 64), read one order ahead;
//  * the orders' (SKU, region, quantity) are read 64 at a time into registers, a chunk
//    ahead, and clamped into range when a chunk becomes current; an order's fields are
//    three readlanes;
//  * the stock row of order i + DIST is loaded into registers when order i starts (a ring
//    of RING row slots), so its memory latency overlaps DIST orders;
//  * a row loaded before an order of the same SKU was decided is stale: the order then
//    takes the row of the most recent such order among the last DIST (still in its slot).
//    The SKUs of the last DIST orders sit in lanes 0..DIST-1 of one register, so the test
//    is one compare; the select runs only on a match;
//  * the chosen warehouse's new stock goes into its lane with a writelane, and to memory
//    with a store from every lane (one address, one value); the load of a later prefetch
//    by that warehouse's lane follows the store in the lane's program order, so it sees it;
//  * an order's action and units shipped go into lane i % 64 of two registers with
//    writelanes and leave 64 at a time.
// Chunks of 64 orders run unrolled, so every slot and lane index is a constant, with no
// branch around a load or a store (a skipped order would leave the compiler unable to
// count the memory operations issued since a prefetch, and it would then wait for every
// outstanding load).  The last, partial chunk runs one order at a time from memory.
constexpr int SER_DIST = 8;
constexpr int SER_RING = 32; // DIST slots ahead, DIST behind for the same-SKU check
static_assert((SER_DIST & (SER_DIST - 1)) == 0 && SER_RING > 2 * SER_DIST && WAVE % SER_RING == 0,
              "ring positions are compile-time constants in a chunk of 64 orders");

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// v with lane L (a compile-time constant) replaced by the wave-uniform value x
template <int L> __device__ __forceinline__ int put_lane(int v, int x)
{
    asm("v_writelane_b32 %0, %1, %2" : "+v"(v) : "s"(x), "i"(L));
    return v;
}

// v with lane l (wave-uniform, written by a scalar instruction) replaced by x; the lane
// select goes in M0 (one scalar register besides M0 per vector instruction)
__device__ __forceinline__ int put_lane_s(int v, int x, int l)
{
    asm("v_writelane_b32 %0, %1, m0" : "+v"(v) : "s"(x), "{m0}"(l));
    return v;
}

// f(integral_constant<int, U>) for U = B .. E-1, in order
template <int B, int E, typename F> __device__ __forceinline__ void static_for(F &f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
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
    const int N = P.N, R = P.R, Km = P.K - 1;
    const int npad = tab_npad<uint16_t>(N);
    const int64_t t0 = P.traj_off[b], t1 = P.traj_off[b + 1];
    const int64_t T = t1 - t0;
    if (T <= 0) return;
    int32_t *xs = state + (int64_t)b * P.K * N;
    // stock rows are addressed by 32-bit byte offsets from xs (the launch checks that a
    // trajectory's K N entries fit): a row's offset is one scalar product
    const char *xbase = (const char *)xs;
    const uint32_t rowb = (uint32_t)N * 4u;
    uint32_t *pairs = (uint32_t *)smem; // [R][64]: key of w = lane, key of w = lane + 64 << 16
    {
        const uint16_t *kb = keys + b * tab_stride<uint16_t>(N, R);
        for (int r = 0; r < R; ++r) {
            const uint32_t lo = lane < npad ? kb[(int64_t)r * npad + lane] : 0xffffu;
            const uint32_t hi = lane + WAVE < npad ? kb[(int64_t)r * npad + lane + WAVE] : 0xffffu;
            pairs[r * WAVE + lane] = lo | (hi << 16);
        }
    }
    // byte offsets of this lane's warehouses in a row (past N: warehouse 0, never chosen)
    const uint32_t l0b = (lane < N ? lane : 0) * 4u, l1b = (lane + WAVE < N ? lane + WAVE : 0) * 4u;
    auto stock = [&](uint32_t off) { return *(const int32_t *)(xbase + off); };
    auto load_chunk = [&](int64_t i, int &k, int &r, int &q) { // raw; past the end: last
        const int64_t t = t0 + i < t1 ? t0 + i : t1 - 1;
        k = P.sku[t];
        r = P.region[t];
        q = P.qty[t];
    };
    int ck, cr, cq, nk, nr, nq;
    load_chunk(lane, ck, cr, cq);
    ck = clampi(ck, 0, Km);
    cr = clampi(cr, 0, R - 1);
    cq = cq < 1 ? 1 : cq;
    load_chunk(WAVE + lane, nk, nr, nq);
    int32_t xa[SER_RING], xb[SER_RING]; // stock of warehouses lane and lane + 64, per slot
    uint32_t ro[SER_RING];              // byte offset of each slot's row (wave-uniform)
#pragma unroll
    for (int u = 0; u < SER_RING; ++u) {
        xa[u] = xb[u] = 0;
        ro[u] = 0;
    }
#pragma unroll
    for (int u = 0; u < SER_DIST; ++u) { // rows of orders 0 .. DIST-1
        ro[u] = (uint32_t)__builtin_amdgcn_readlane(ck, u) * rowb;
        xa[u] = stock(ro[u] + l0b);
        xb[u] = stock(ro[u] + l1b);
    }
    __syncthreads(); // the key pairs
    int recent = -1; // lane j < DIST: SKU of the last order in ring position j
    uint32_t kp = pairs[__builtin_amdgcn_readlane(cr, 0) * WAVE + lane]; // next order's keys
    int act = LOST, shp = 0;
    // the decision for one order from its row (byte offset rof) and key pair; returns
    // (action, shipped).  Without branches: a lost sale (no warehouse with stock) stores
    // warehouse 0's stock back unchanged, so every order issues exactly one store and the
    // compiler can count the memory operations between a prefetch and its use.
    auto decide = [&](uint32_t rof, int q, int32_t &x0v, int32_t &x1v, uint32_t kk, int &a,
                      int &sh) {
        const uint32_t k0 = x0v > 0 ? (kk & 0xffffu) : 0xffffu;
        const uint32_t k1 = x1v > 0 ? (kk >> 16) : 0xffffu;
        const uint32_t best = wave_min_u32(k0 < k1 ? k0 : k1);
        const bool found = best != 0xffffu;
        const int w = found ? (int)(best & 0xffu) : 0; // the warehouse whose stock is written
        const int own = w & (WAVE - 1);
        const bool hi = w >= WAVE;
        const int32_t xv0 = __builtin_amdgcn_readlane(x0v, own);
        const int32_t xv1 = __builtin_amdgcn_readlane(x1v, own);
        const int32_t xv = hi ? xv1 : xv0;
        sh = found ? (q < xv ? q : xv) : 0;
        const int32_t nv = xv - sh;
        x0v = put_lane_s(x0v, hi ? xv0 : nv, own);
        x1v = put_lane_s(x1v, hi ? nv : xv1, own);
        *(int32_t *)((char *)xs + (rof + (uint32_t)w * 4u)) = nv;
        a = found ? w : LOST;
    };
    const int64_t full = T - T % WAVE;
    for (int64_t g = 0; g < full; g += WAVE) {
        if (g > 0) { // the next chunk becomes current; load the one after it
            ck = clampi(nk, 0, Km);
            cr = clampi(nr, 0, R - 1);
            cq = nq < 1 ? 1 : nq;
            load_chunk(g + WAVE + lane, nk, nr, nq);
        }
        auto order = [&](auto uc) {
            constexpr int u = decltype(uc)::value;
            constexpr int s = u & (SER_RING - 1), pos = u & (SER_DIST - 1);
            // prefetch first (its address math fills the reduction's wait states): the row
            // of order i + DIST, of the next chunk for the last DIST orders
            {
                const int kf = u + SER_DIST < WAVE
                                   ? __builtin_amdgcn_readlane(ck, (u + SER_DIST) & (WAVE - 1))
                                   : clampi(__builtin_amdgcn_readlane(nk, (u + SER_DIST) & (WAVE - 1)),
                                            0, Km);
                constexpr int sf = (u + SER_DIST) & (SER_RING - 1);
                ro[sf] = (uint32_t)kf * rowb;
                xa[sf] = stock(ro[sf] + l0b);
                xb[sf] = stock(ro[sf] + l1b);
            }
            const int k = __builtin_amdgcn_readlane(ck, u);
            const int q = __builtin_amdgcn_readlane(cq, u);
            const uint32_t kk = kp;
            // the next order's key pair (its region: this chunk, or the next one's first)
            const int rn = u + 1 < WAVE ? __builtin_amdgcn_readlane(cr, (u + 1) & (WAVE - 1))
                                        : clampi(__builtin_amdgcn_readlane(nr, 0), 0, R - 1);
            kp = pairs[rn * WAVE + lane];
            // the row: this slot's prefetch, unless one of the last DIST orders (all decided
            // after the prefetch was issued) has the same SKU: then the most recent of them
            // holds the current row
            int32_t x0v = xa[s], x1v = xb[s];
            const uint64_t hit = __ballot(recent == k) & ((1ull << SER_DIST) - 1);
            if (__builtin_expect(hit != 0, 0)) {
#pragma unroll
                for (int d = SER_DIST; d >= 1; --d) {
                    if ((hit >> ((u - d) & (SER_DIST - 1))) & 1) {
                        x0v = xa[(u - d) & (SER_RING - 1)];
                        x1v = xb[(u - d) & (SER_RING - 1)];
                    }
                }
            }
            recent = put_lane<pos>(recent, k);
            int a, sh;
            decide(ro[s], q, x0v, x1v, kk, a, sh);
            xa[s] = x0v;
            xb[s] = x1v;
            act = put_lane<u>(act, a);
            shp = put_lane<u>(shp, sh);
        };
        static_for<0, WAVE>(order);
        actions[t0 + g + lane] = act;
        if (shipped) shipped[t0 + g + lane] = shp;
    }
    if (full < T) { // the last, partial chunk, one order at a time with rows from memory
        if (full > 0) {
            ck = clampi(nk, 0, Km);
            cr = clampi(nr, 0, R - 1);
            cq = nq < 1 ? 1 : nq;
        }
        for (int u = 0; u < (int)(T - full); ++u) {
            const int k = __builtin_amdgcn_readlane(ck, u);
            const int r = __builtin_amdgcn_readlane(cr, u);
            const int q = __builtin_amdgcn_readlane(cq, u);
            const uint32_t rof = (uint32_t)k * rowb;
            int32_t x0v = stock(rof + l0b), x1v = stock(rof + l1b);
            int a, sh;
            decide(rof, q, x0v, x1v, pairs[r * WAVE + lane], a, sh);
            act = lane == u ? a : act;
            shp = lane == u ? sh : shp;
        }
        if (lane < T - full) {
            actions[t0 + full + lane] = act;
            if (shipped) shipped[t0 + full + lane] = shp;
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
    const size_t tab_b = (size_t)P.R * WAVE * 4; // key pairs
    if (P.N <= 2 * WAVE && tab_b <= 64 * 1024 && (int64_t)P.K * P.N * 4 <= INT32_MAX)
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

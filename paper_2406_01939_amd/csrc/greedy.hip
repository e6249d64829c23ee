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

// key[b][r][w] = (position of w in region r's increasing (cost[b][w][r], w) order) << S
// | w.  One workgroup per row (b, r): the row's costs are staged in LDS, then one thread
// per w counts the warehouses that precede it.  Row padding is all-ones.
template <typename KeyT>
__global__ __launch_bounds__(256) void k_keys(Prob P, KeyT *keys)
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
        for (int w = threadIdx.x; w < npad; w += blockDim.x) {
            if (w >= N) {
                row[w] = (KeyT)~(KeyT)0;
                continue;
            }
            const int32_t cw = cs[w];
            uint32_t q = 0;
            for (int v = 0; v < N; ++v) {
                const int32_t cv = cs[v];
                q += (cv < cw) || (cv == cw && v < w);
            }
            row[w] = (KeyT)((q << key_shift<KeyT>()) | (uint32_t)w);
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

hipError_t setup_pos(const Prob &P, void *keys, hipStream_t st)
{
    int64_t g = (int64_t)P.n_traj * P.R; // one workgroup per row
    g = g < 1 ? 1 : (g > 8192 ? 8192 : g);
    const int threads = P.N <= 128 ? 128 : 256;
    if (keys16(P.N))
        hipLaunchKernelGGL(k_keys<uint16_t>, dim3((unsigned)g), dim3(threads), 0, st, P,
                           (uint16_t *)keys);
    else
        hipLaunchKernelGGL(k_keys<uint32_t>, dim3((unsigned)g), dim3(threads), 0, st, P,
                           (uint32_t *)keys);
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

// Picard iteration for the One Warehouse Multi-Retailer (OWMR) inventory problem (the
// appendix's inventory-control extension): one central warehouse under an (s, S) rule,
// N retailers ordering up to their level S_n when their stock after the demand is at most
// s_n (within capacity c_n); an order of step t is a demand d_t at retailer n_t, the
// retailer receives min(q, x_0), the central stock becomes S after a reset, else
// (x_0 - q)^+.  The action of a step is (q, reset); a cached reset is the decision to
// order up to S.
//
// Processes are retailers (the appendix's allocation T_n).  In a pass a retailer's own
// stock changes only at its own steps, so its lane keeps it in a register; the central
// stock it sees at its step t follows the previous pass's cached actions since its own
// previous step a-1: after the last cached reset r in [a, t) it is S minus the cached
// orders of steps r+1 .. t-1, else the stock after its previous step minus the cached
// orders of steps a .. t-1, both clamped at zero (clamped subtractions compose).  With
//   V[t] = reset_t * 2^40 + q_t   (the cache, time order)   and   S = exclusive scan of V,
// the low 40 bits of S[t] are the orders before t and the high bits the resets before t;
// the list of resets (their times and the order sums just after them) comes from one
// scatter.  A pass is: scan V -> S (out of place), the reset list, the retailer walk
// (which rewrites V in place and counts changes), the pass end.
#include "pk_internal.h"

namespace pk {

constexpr int OW_SHIFT = 40;
constexpr int64_t OW_QMASK = ((int64_t)1 << OW_SHIFT) - 1;
constexpr int OW_DIST = 8; // steps a retailer lane loads ahead

namespace {

// The retailer policy: order at stock x (before the demand) for demand d.
__device__ __forceinline__ int64_t ow_order(int64_t x, int64_t d, int32_t s_n, int32_t S_n,
                                            int32_t c_n)
{
    const int64_t p = x > d ? x - d : 0;
    const int64_t level = S_n < c_n ? S_n : c_n;
    return p <= s_n && level > p ? level - p : 0;
}

// Sorted positions (by retailer, then time) from the stable sort: seg[n] counts.
__global__ void k_ow_count(OwmrDev P, int32_t *cnt, int32_t *err)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < P.T; t += stride) {
        const int n = P.retailer[t];
        if (n < 0 || n >= P.N || P.demand[t] < 0) {
            atomicOr(err, 1);
            continue;
        }
        atomicAdd(&cnt[n], 1);
    }
}

// Initial cache (empty: no order, no reset) or the caller's, packed in time order.
__global__ void k_ow_init(OwmrDev P, const int32_t *iq, const int32_t *ir, int64_t *V)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < P.T; t += stride)
        V[t] = iq ? (((int64_t)(ir[t] != 0) << OW_SHIFT) + (iq[t] > 0 ? iq[t] : 0)) : 0;
}

// The reset list: the j-th cached reset at time t gets rq[j] = orders up to and including
// t (the low bits of S[t] + V[t]), the base of the central stock after it.
__global__ void k_ow_resets(OwmrDev P, const OwmrCtl *ctl, const int64_t *V, const int64_t *S,
                            int64_t *rq)
{
    if (ctl->done) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < P.T; t += stride) {
        const int64_t v = V[t];
        if (v >> OW_SHIFT) {
            const int64_t s = S[t];
            rq[s >> OW_SHIFT] = (s & OW_QMASK) + (v & OW_QMASK);
        }
    }
}

// One lane per retailer walks its steps in time order (sorted positions seg[n] ..
// seg[n+1]: time index perm[i], demand sd[i]).  Loads run in two stages ahead of the step
// being decided: the time index and demand 2 DIST steps ahead (sequential per lane), then
// the scan value and the old cache of the step DIST ahead (at that time index), then the
// reset base of the step DIST / 2 ahead (at its count of resets).  The
// groups of DIST steps that every lane of the wave has run without a per-step test, their
// look-ahead loads clamped into the lane's range, so the compiler counts the loads between
// a prefetch and its use exactly; the rest run with the test.  Lanes past the last
// retailer shadow it and write to the sink.  REC: write each pass's cache to `caches`.
template <bool REC>
__global__ __launch_bounds__(64) void k_ow_walk(OwmrDev P, OwmrCtl *ctl, const int32_t *perm,
                                                const int32_t *sd, const int32_t *seg,
                                                const int64_t *S, const int64_t *rq, int64_t *V,
                                                int64_t *final_x0v, int32_t *final_x,
                                                int64_t *caches, int64_t *sink)
{
    if (ctl->done) return;
    const int lane = threadIdx.x;
    const int n0 = blockIdx.x * 64 + lane;
    const bool valid = n0 < P.N;
    const int n = valid ? n0 : P.N - 1;
    unsigned long long changed = 0;
    const int32_t lo = seg[n], hi = seg[n + 1];
    const int32_t last = hi > lo ? hi - 1 : lo; // a position of the lane's range (or lo)
    const int32_t s_n = P.s_ret[n], S_n = P.S_ret[n], c_n = P.cap[n];
    int64_t x = P.x_init[n];
    int64_t x0v = P.x0_init; // central stock after this retailer's previous step
    int64_t s_a = 0;         // S at a = previous step + 1 (orders and resets before a)
    int32_t at[OW_DIST], ad[OW_DIST];                  // stage A: i + 2 DIST
    int32_t bt[OW_DIST], bd[OW_DIST];                  // stage B: i + DIST
    int64_t bs[OW_DIST], bv[OW_DIST];
    int64_t rqv[OW_DIST]; // stage C: the reset base of the step DIST / 2 ahead
    const bool any = hi > lo;
#pragma unroll
    for (int k = 0; k < OW_DIST; ++k) {
        const int32_t i = lo + k, j = lo + OW_DIST + k;
        bt[k] = any ? perm[i < hi ? i : last] : 0;
        bd[k] = any ? sd[i < hi ? i : last] : 0;
        at[k] = any ? perm[j < hi ? j : last] : 0;
        ad[k] = any ? sd[j < hi ? j : last] : 0;
    }
#pragma unroll
    for (int k = 0; k < OW_DIST; ++k) {
        bs[k] = any ? S[bt[k]] : 0;
        bv[k] = any ? V[bt[k]] : 0;
    }
    // rq index of a step: its last cached reset before it (rq[0] when there is none: unused)
    auto rq_at = [&](int64_t s_t) {
        const int64_t c = s_t >> OW_SHIFT;
        return rq[c > 0 ? c - 1 : 0];
    };
#pragma unroll
    for (int k = 0; k < OW_DIST; ++k) rqv[k] = k < OW_DIST / 2 ? rq_at(bs[k]) : 0;
    // one step (step i of the lane, slot k of its group)
    auto step = [&](int32_t i, int k) {
        // stage C: the reset base of step i + DIST/2, whose S value arrived DIST/2 steps ago
        const int kc = (k + OW_DIST / 2) & (OW_DIST - 1);
        const int64_t rq_t = rqv[k];
        rqv[kc] = rq_at(bs[kc]);
        const int32_t t = bt[k];
        const int64_t d = bd[k], s_t = bs[k], v_old = bv[k];
        // stage B takes over stage A's step (DIST ahead) and loads its values; stage A
        // loads the step 2 DIST ahead (clamped into the range: past it, unused)
        const int32_t ia = i + 2 * OW_DIST < hi ? i + 2 * OW_DIST : last;
        bt[k] = at[k];
        bd[k] = ad[k];
        bs[k] = S[at[k]];
        bv[k] = V[at[k]];
        at[k] = perm[ia];
        ad[k] = sd[ia];
        // the central stock at t: resets and orders of the others' steps since a
        const int64_t c_t = s_t >> OW_SHIFT, c_a = s_a >> OW_SHIFT;
        const int64_t v = c_t > c_a ? P.S0 - ((s_t & OW_QMASK) - rq_t)
                                    : x0v - ((s_t & OW_QMASK) - (s_a & OW_QMASK));
        const int64_t x0 = v > 0 ? v : 0;
        const int64_t q = ow_order(x, d, s_n, S_n, c_n);
        const int reset = x0 - q <= P.s0;
        const int64_t v_new = ((int64_t)reset << OW_SHIFT) + q;
        changed += valid && v_new != v_old;
        *(valid ? &V[t] : &sink[lane]) = v_new;
        if constexpr (REC) *(valid ? &caches[t] : &sink[lane]) = v_new;
        const int64_t p = x > d ? x - d : 0;
        x = p + (q < x0 ? q : x0);
        x0v = reset ? P.S0 : (x0 > q ? x0 - q : 0);
        s_a = s_t + v_old; // S at t + 1 in the previous pass's cache
    };
    // groups every lane runs in full (a wave-uniform count)
    int32_t g_all = (hi - lo) / OW_DIST;
    for (int o = 32; o > 0; o >>= 1) {
        const int32_t other = __shfl_xor(g_all, o, 64);
        g_all = other < g_all ? other : g_all;
    }
    g_all = __builtin_amdgcn_readfirstlane(g_all);
    int32_t i0 = lo;
    for (int32_t g = 0; g < g_all; ++g, i0 += OW_DIST) {
#pragma unroll
        for (int k = 0; k < OW_DIST; ++k) step(i0 + k, k);
    }
    for (; i0 < hi; i0 += OW_DIST) {
#pragma unroll
        for (int k = 0; k < OW_DIST; ++k)
            if (i0 + k < hi) step(i0 + k, k); // (the last groups' tails: per lane)
    }
    if (valid) {
        final_x[n] = (int32_t)x;
        final_x0v[n] = x0v;
    }
    // changes of the wave, one atomic
    for (int o = 32; o > 0; o >>= 1) changed += __shfl_xor(changed, o, 64);
    if (threadIdx.x == 0 && changed) atomicAdd(&ctl->changed, changed);
}

__global__ void k_ow_gather(const int32_t *perm, const int32_t *src, int32_t *dst, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = src[perm[i]];
}

__global__ void k_ow_iota(int32_t *v, const int32_t *src, int32_t *keys, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        v[i] = (int32_t)i;
        keys[i] = src[i];
    }
}

__global__ void k_ow_pass_end(OwmrCtl *ctl)
{
    if (threadIdx.x != 0 || blockIdx.x != 0 || ctl->done) return;
    const int p = ctl->pass;
    ctl->changed_log[(p - 1) & 7] = ctl->changed;
    if (ctl->changed == 0) {
        ctl->done = 1;
        ctl->passes_done = p;
    } else if (p >= ctl->max_passes) {
        ctl->done = 2;
        ctl->passes_done = p;
    }
    ctl->changed = 0;
    ctl->pass = p + 1;
}

__global__ void k_ow_ctl_init(OwmrCtl *ctl, int32_t max_passes)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    ctl->pass = 1;
    ctl->done = 0;
    ctl->passes_done = 0;
    ctl->max_passes = max_passes;
    ctl->error = 0;
    ctl->changed = 0;
    for (int i = 0; i < 8; ++i) ctl->changed_log[i] = 0;
}

// Outputs in time order from the packed cache.
__global__ void k_ow_unpack(OwmrDev P, const int64_t *V, int32_t *q, int32_t *reset)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < P.T; t += stride) {
        const int64_t v = V[t];
        q[t] = (int32_t)(v & OW_QMASK);
        reset[t] = (int32_t)(v >> OW_SHIFT);
    }
}

// The serial sweep: one wave; lane 0 takes the steps in time order with the retailers'
// stock in LDS and the central stock in a register; the steps' retailer and demand are
// read 64 at a time, a chunk ahead, by the whole wave.
__global__ __launch_bounds__(64) void k_ow_serial(OwmrDev P, int32_t *q_out, int32_t *r_out,
                                                  int64_t *final_x0, int32_t *final_x,
                                                  unsigned long long *resets)
{
    extern __shared__ int32_t xs[];
    const int lane = threadIdx.x;
    for (int n = lane; n < P.N; n += 64) xs[n] = P.x_init[n];
    __syncthreads();
    int64_t x0 = P.x0_init;
    unsigned long long R = 0;
    int cr = 0, cd = 0, nr = 0, nd = 0;
    if (lane < P.T) { cr = P.retailer[lane]; cd = P.demand[lane]; }
    if (64 + lane < P.T) { nr = P.retailer[64 + lane]; nd = P.demand[64 + lane]; }
    int sq = 0, sr = 0; // lane j: the outputs of step c + j
    for (int64_t c = 0; c < P.T; c += 64) {
        const int m = P.T - c < 64 ? (int)(P.T - c) : 64;
        for (int j = 0; j < m; ++j) {
            const int n = __builtin_amdgcn_readlane(cr, j);
            const int64_t d = __builtin_amdgcn_readlane(cd, j);
            int qv = 0, rv = 0;
            if (lane == 0) {
                const int64_t x = xs[n];
                const int64_t q = ow_order(x, d, P.s_ret[n], P.S_ret[n], P.cap[n]);
                const int reset = x0 - q <= P.s0;
                const int64_t p = x > d ? x - d : 0;
                xs[n] = (int32_t)(p + (q < x0 ? q : x0));
                x0 = reset ? P.S0 : (x0 > q ? x0 - q : 0);
                R += reset;
                qv = (int)q;
                rv = reset;
            }
            const int bq = __builtin_amdgcn_readlane(qv, 0), br = __builtin_amdgcn_readlane(rv, 0);
            if (lane == j) {
                sq = bq;
                sr = br;
            }
        }
        if (c + lane < P.T) {
            q_out[c + lane] = sq;
            r_out[c + lane] = sr;
        }
        cr = nr;
        cd = nd;
        if (c + 128 + lane < P.T) {
            nr = P.retailer[c + 128 + lane];
            nd = P.demand[c + 128 + lane];
        }
    }
    __syncthreads();
    for (int n = lane; n < P.N; n += 64) final_x[n] = xs[n];
    if (lane == 0) {
        *final_x0 = x0;
        *resets = R;
    }
}

// Per-retailer checks: capacity, starting stock within it, levels; orders fit the packed
// cache (T c_n < 2^40).
__global__ void k_ow_check(OwmrDev P, int32_t *err)
{
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < P.N; n += gridDim.x * blockDim.x) {
        const int64_t c = P.cap[n];
        if (c < 0 || P.x_init[n] < 0 || P.x_init[n] > c || P.S_ret[n] < 0 ||
            (int64_t)c * (P.T > 0 ? P.T : 1) >= ((int64_t)1 << OW_SHIFT))
            atomicOr(err, 1);
    }
}

__global__ void k_ow_zero(int32_t *a, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0;
}

inline unsigned grid_for(int64_t n, int64_t cap_blocks = 8192)
{
    int64_t g = (n + 255) / 256;
    return (unsigned)(g < 1 ? 1 : (g > cap_blocks ? cap_blocks : g));
}

} // namespace

size_t owmr_radix_tmp(int64_t T) { return radix_tmp_bytes(T); }

hipError_t owmr_launch_setup(const OwmrDev &P, int32_t *keys, int32_t *keys_alt, int32_t *vals,
                             int32_t *vals_alt, void *rtmp, int32_t *cnt, void *stmp,
                             int32_t *sd, int32_t *err, int32_t **perm, hipStream_t st)
{
    hipError_t e = hipSuccess;
    hipLaunchKernelGGL(k_ow_zero, dim3(grid_for((int64_t)P.N + 1)), dim3(256), 0, st, cnt,
                       (int64_t)P.N + 1);
    hipLaunchKernelGGL(k_ow_zero, dim3(1), dim3(64), 0, st, err, (int64_t)1);
    hipLaunchKernelGGL(k_ow_check, dim3(grid_for(P.N)), dim3(256), 0, st, P, err);
    hipLaunchKernelGGL(k_ow_count, dim3(grid_for(P.T)), dim3(256), 0, st, P, cnt, err);
    if ((e = scan_i32_excl(cnt, (int64_t)P.N + 1, stmp, st)) != hipSuccess) return e;
    *perm = vals;
    if (P.T == 0) return hipGetLastError();
    hipLaunchKernelGGL(k_ow_iota, dim3(grid_for(P.T)), dim3(256), 0, st, vals, P.retailer, keys,
                       P.T);
    int bits = 1;
    while ((1 << bits) < P.N) ++bits;
    bool in_alt = false;
    if ((e = radix_sort_pairs(keys, vals, keys_alt, vals_alt, P.T, bits, rtmp, st, &in_alt)) !=
        hipSuccess)
        return e;
    *perm = in_alt ? vals_alt : vals;
    hipLaunchKernelGGL(k_ow_gather, dim3(grid_for(P.T)), dim3(256), 0, st, *perm, P.demand, sd,
                       P.T);
    return hipGetLastError();
}

hipError_t owmr_launch_init(const OwmrDev &P, const int32_t *iq, const int32_t *ir, int64_t *V,
                            OwmrCtl *ctl, int32_t max_passes, hipStream_t st)
{
    hipLaunchKernelGGL(k_ow_ctl_init, dim3(1), dim3(64), 0, st, ctl, max_passes);
    hipLaunchKernelGGL(k_ow_init, dim3(grid_for(P.T)), dim3(256), 0, st, P, iq, ir, V);
    return hipGetLastError();
}

hipError_t owmr_launch_pass(const OwmrDev &P, OwmrCtl *ctl, const int32_t *perm, const int32_t *sd,
                            const int32_t *seg, int64_t *V, int64_t *S, int64_t *rq, void *stmp,
                            int64_t *fx0v, int32_t *fx, int64_t *caches, int64_t *sink,
                            hipStream_t st)
{
    if (P.T > 0) {
        hipError_t e = scan_i64_to(V, S, P.T, false, stmp, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_ow_resets, dim3(grid_for(P.T)), dim3(256), 0, st, P, ctl, V, S, rq);
    }
    if (caches)
        hipLaunchKernelGGL(k_ow_walk<true>, dim3((unsigned)((P.N + 63) / 64)), dim3(64), 0, st, P,
                           ctl, perm, sd, seg, S, rq, V, fx0v, fx, caches, sink);
    else
        hipLaunchKernelGGL(k_ow_walk<false>, dim3((unsigned)((P.N + 63) / 64)), dim3(64), 0, st, P,
                           ctl, perm, sd, seg, S, rq, V, fx0v, fx, caches, sink);
    hipLaunchKernelGGL(k_ow_pass_end, dim3(1), dim3(64), 0, st, ctl);
    return hipGetLastError();
}

hipError_t owmr_launch_unpack(const OwmrDev &P, const int64_t *V, int32_t *q, int32_t *r,
                              hipStream_t st)
{
    if (P.T == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ow_unpack, dim3(grid_for(P.T)), dim3(256), 0, st, P, V, q, r);
    return hipGetLastError();
}

hipError_t owmr_launch_serial(const OwmrDev &P, int32_t *q, int32_t *r, int64_t *fx0, int32_t *fx,
                              unsigned long long *resets, hipStream_t st)
{
    hipLaunchKernelGGL(k_ow_serial, dim3(1), dim3(64), sizeof(int32_t) * (size_t)P.N, st, P, q, r,
                       fx0, fx, resets);
    return hipGetLastError();
}

} // namespace pk

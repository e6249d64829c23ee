// Device side of the policy-gradient loop around the rollout (Section 4.2 trains the
// policy with Adam on rolled-out trajectories): per-step REINFORCE advantages computed
// from the rollout's actions, and the Adam update of the parameter pack.
//
// Advantages.  The reward of step t is the chosen warehouse's margin on what it ships,
// r_t = (revenue - cost[a_t][region_t]) * shipped_t, and 0 for a lost sale (the FO model
// of Section 3 earns the chosen node's reward, nothing when the order is not served; the
// margin form is that reward with a per-unit revenue).  A_t is the reward-to-go of step t
// minus its mean over the trajectory.  Rewards, reward-to-go and the per-trajectory sum
// of reward-to-go are exact int64 (the host bounds |r_t| so that no sum can overflow);
// the one rounding step is the final double subtraction, so the result does not depend
// on the order in which the device adds.
#include "pk_internal.h"

namespace pk {

namespace {

constexpr int ADV_THREADS = 256;
constexpr int ADV_ITEMS = 8;
constexpr int ADV_TILE = ADV_THREADS * ADV_ITEMS;
constexpr int ADAM_THREADS = 256;

// Trajectory of flat order i: the largest b with offs[b] <= i.  Offsets are
// nondecreasing, so an empty trajectory (offs[b] == offs[b+1]) is never returned for an
// order it does not own.
__device__ __forceinline__ int traj_of(const int64_t *offs, int n_traj, int64_t i)
{
    int lo = 0, hi = n_traj - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (offs[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Rewards r_t into rew[], and per trajectory the weighted sum sum_u r_u * (u - lo + 1),
// which equals the sum of the reward-to-go over the trajectory.  One tile of ADV_TILE
// consecutive orders per workgroup; a tile inside one trajectory adds its sum with one
// atomic, a tile that straddles trajectories adds per order.
__global__ __launch_bounds__(ADV_THREADS) void k_rewards(
    const int64_t *offs, int n_traj, int N, int R, const int32_t *region, const int32_t *actions,
    const int32_t *shipped, const int32_t *cost, int32_t revenue, int64_t rlim, int64_t total,
    int64_t *rew, unsigned long long *wsum, int32_t *err)
{
    __shared__ unsigned long long red[ADV_THREADS / WAVE];
    const int64_t base = (int64_t)blockIdx.x * ADV_TILE;
    const int64_t last = min(base + ADV_TILE, total) - 1;
    const int b0 = traj_of(offs, n_traj, base);
    const bool one = traj_of(offs, n_traj, last) == b0;
    const int64_t lo0 = offs[b0];
    int64_t part = 0;
    for (int k = 0; k < ADV_ITEMS; ++k) {
        const int64_t i = base + (int64_t)k * ADV_THREADS + threadIdx.x;
        if (i >= total) break;
        const int b = one ? b0 : traj_of(offs, n_traj, i);
        const int32_t a = actions[i];
        const int32_t s = shipped[i];
        int64_t r = 0;
        if (a < -1 || a >= N || s < 0) {
            atomicOr(err, 1);
        } else if (a >= 0) {
            const int32_t reg = region[i];
            if (reg < 0 || reg >= R) {
                atomicOr(err, 1);
            } else {
                const int64_t margin = (int64_t)revenue - cost[((int64_t)b * N + a) * R + reg];
                const uint64_t am = (uint64_t)(margin < 0 ? -margin : margin);
                // |r| = am * s > rlim, with the product exact (am < 2^32, s < 2^31)
                if (am * (uint64_t)s > (uint64_t)rlim) atomicOr(err, 2);
                else r = margin * s;
            }
        }
        rew[i] = r;
        const int64_t w = r * (i - (one ? lo0 : offs[b]) + 1);
        if (one) part += w;
        else if (w != 0) atomicAdd(&wsum[b], (unsigned long long)w);
    }
    if (!one) return;
    // two's-complement addition is exact and order-free, so unsigned atomics sum int64
    unsigned long long v = (unsigned long long)part;
    for (int d = WAVE / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, WAVE);
    if (__lane_id() == 0) red[threadIdx.x / WAVE] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
        for (int w = 0; w < ADV_THREADS / WAVE; ++w) s += red[w];
        if (s != 0) atomicAdd(&wsum[b0], s);
    }
}

// A_t = rtg_t - mean_b(rtg), from the inclusive prefix P of the rewards over the whole
// batch: rtg_t = P[hi-1] - P[t-1].  Also the trajectory's return (rtg at its first order).
__global__ __launch_bounds__(ADV_THREADS) void k_advantages(
    const int64_t *offs, int n_traj, const int64_t *P, const unsigned long long *wsum,
    int64_t total, float *adv, int64_t *ret)
{
    const int64_t i = (int64_t)blockIdx.x * ADV_THREADS + threadIdx.x;
    if (i >= total) return;
    const int b = traj_of(offs, n_traj, i);
    const int64_t lo = offs[b], hi = offs[b + 1];
    const int64_t before = i > 0 ? P[i - 1] : 0;
    const int64_t rtg = P[hi - 1] - before;
    const double mean = (double)(int64_t)wsum[b] / (double)(hi - lo);
    adv[i] = (float)((double)rtg - mean);
    if (ret && i == lo) ret[b] = rtg;
}

// Adam (Kingma and Ba, Algorithm 1) on a flat float pack, in float32:
//   m <- b1 m + (1-b1) g,  v <- b2 v + (1-b2) g^2,
//   theta <- theta + dir * lr * (m / bc1) / (sqrt(v / bc2) + eps),  bc_i = 1 - b_i^step,
// dir = +1 to ascend the objective (the REINFORCE surrogate), -1 to descend.
__global__ __launch_bounds__(ADAM_THREADS) void k_adam(float *p, const float *g, float *m,
                                                       float *v, int64_t n, AdamCoef c)
{
    const int64_t i = (int64_t)blockIdx.x * ADAM_THREADS + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = c.b1 * m[i] + c.omb1 * gi;
    const float vi = c.b2 * v[i] + c.omb2 * (gi * gi);
    m[i] = mi;
    v[i] = vi;
    const float step = c.lr * (mi / c.bc1) / (sqrtf(vi / c.bc2) + c.eps);
    p[i] = p[i] + c.dir * step;
}

} // namespace

size_t advantages_ws_bytes(int64_t total, int n_traj)
{
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    return al((size_t)(n_traj + 1) * 8) + al((size_t)std::max<int64_t>(total, 1) * 8) +
           al((size_t)n_traj * 8) + al(4) + al(scan_tmp_bytes(total)) + 256;
}

hipError_t launch_advantages(const int64_t *offs_dev, int n_traj, int N, int R, int64_t total,
                             const int32_t *region, const int32_t *actions,
                             const int32_t *shipped, const int32_t *cost, int32_t revenue,
                             int64_t rlim, int64_t *rew, unsigned long long *wsum, int32_t *err,
                             void *scan_tmp, float *adv, int64_t *ret, hipStream_t st)
{
    if (total <= 0) return hipSuccess;
    const int64_t tiles = (total + ADV_TILE - 1) / ADV_TILE;
    hipLaunchKernelGGL(k_rewards, dim3((unsigned)tiles), dim3(ADV_THREADS), 0, st, offs_dev,
                       n_traj, N, R, region, actions, shipped, cost, revenue, rlim, total, rew,
                       wsum, err);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = scan_i64(rew, total, true, scan_tmp, st)) != hipSuccess) return e;
    const int64_t blocks = (total + ADV_THREADS - 1) / ADV_THREADS;
    hipLaunchKernelGGL(k_advantages, dim3((unsigned)blocks), dim3(ADV_THREADS), 0, st, offs_dev,
                       n_traj, rew, wsum, total, adv, ret);
    return hipGetLastError();
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, int64_t n,
                       const AdamCoef &c, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + ADAM_THREADS - 1) / ADAM_THREADS;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(ADAM_THREADS), 0, st, p, g, m, v, n, c);
    return hipGetLastError();
}

} // namespace pk

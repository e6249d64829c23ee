// Learned softmax policy kernels: the MLP scorer on MFMA, the Picard run walk, the serial
// sweep and a diagnostic scorer.
//
// Policy (learned fulfillment policy, trained by policy gradient in Section 4.2): per
// (order, warehouse) row the features [cost[w][r], log1p(x[w]), E[r][0..15]] go through
// h1 = relu(W1 f + b1), h2 = relu(W2 h1 + b2), s = w3 . h + b3 (h = h2, or h1 with one
// hidden layer); the action is argmax over warehouses with stock of s_w + G(t, traj, w)
// (lowest index on exact ties), G a Gumbel variate; this samples softmax(s) over the
// warehouses with stock.  The noise is part of the order's disturbance (Section 2).
//
// Scorer: 16 rows (warehouses of one order) per wave step, in transposed form so that a
// layer's MFMA output registers are directly the next layer's MFMA input:
//   H1^T[64 x 16] = W1[64 x 20] F^T[20 x 16]    (features padded 18 -> 20)
//   H2^T[64 x 16] = W2[64 x 64] H1^T[64 x 16]
// with v_mfma_f32_16x16x4f32 (A: lane l holds A[l%16][l/16]; B: lane l holds
// B[l/16][l%16]; D: lane l, register v holds D[4(l/16)+v][l%16]).  Lane l keeps hidden
// units 16t + 4(l/16) + v of row l%16, so layer 2 sums its k dimension in the order
// h = 16(s/4) + 4(l/16) + s%4 over its 16 steps s; W2's A operand is loaded in that
// order.  The accumulation order of every row's dot products is fixed, so a row's score
// does not depend on which other rows share its tile (the walk and the serial sweep
// produce bit-identical scores).
#include <math.h>

#include "pk_internal.h"

namespace pk {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- Philox4x32-10 (SC'11)
// Round: 32x32->64 products of counter words 0 and 2 with the round multipliers; new
// counter (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)); the key is
// bumped by the Weyl constants between rounds.
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Gumbel variate of (order t of trajectory traj, warehouse w): counter (t, traj, w/4, 0),
// word w%4; U = ((u >> 9) + 0.5) 2^-23 (exact in binary32); G = -log(-log U).
__device__ __forceinline__ float gumbel(uint64_t seed, uint32_t traj, uint32_t t, uint32_t w)
{
    const uint4 o = philox10(make_uint4(t, traj, w >> 2, 0u), (uint32_t)seed,
                             (uint32_t)(seed >> 32));
    const uint32_t u = (w & 3) == 0 ? o.x : (w & 3) == 1 ? o.y : (w & 3) == 2 ? o.z : o.w;
    const float U = ((float)(u >> 9) + 0.5f) * (1.0f / 8388608.0f);
    return -logf(-logf(U));
}

// ---------------------------------------------------------------- MFMA scorer
struct MlpLane {
    float a1[20]; // layer 1 A operands, index t*5 + s
    float a2[64]; // layer 2 A operands, index t*16 + s
    float b1[16], b2[16], w3[16]; // index t*4 + v (hidden 16t + 4g + v)
    float b3;
    const float *E; // [R][16] in global memory
    int two;        // two hidden layers
};

__device__ __forceinline__ void load_mlp(MlpLane &m, const float *params, int R, int layers)
{
    const int l = __lane_id(), i = l & 15, g = l >> 4;
    const float *E = params;
    const float *W1 = E + (int64_t)R * 16;
    const float *b1 = W1 + 64 * 18;
    const float *W2 = b1 + 64;
    const float *b2 = W2 + 64 * 64;
    const float *w3 = layers == 2 ? b2 + 64 : b1 + 64;
    m.E = E;
    m.two = layers == 2;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int s = 0; s < 5; ++s) {
            const int k = 4 * s + g;
            m.a1[t * 5 + s] = k < 18 ? W1[(16 * t + i) * 18 + k] : 0.0f;
        }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            m.b1[t * 4 + v] = b1[16 * t + 4 * g + v];
            m.w3[t * 4 + v] = w3[16 * t + 4 * g + v];
            m.b2[t * 4 + v] = layers == 2 ? b2[16 * t + 4 * g + v] : 0.0f;
        }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const int h = 16 * (s >> 2) + 4 * g + (s & 3);
            m.a2[t * 16 + s] = layers == 2 ? W2[(16 * t + i) * 64 + h] : 0.0f;
        }
    m.b3 = w3[64];
}

// Feature k = 4s + g of row l%16 for this lane: [cost, log1p x, E[r][0..15], 0, 0].
__device__ __forceinline__ void lane_features(float f[5], float cost, float lx, const float *Er)
{
    const int g = __lane_id() >> 4;
#pragma unroll
    for (int s = 0; s < 5; ++s) {
        const int k = 4 * s + g;
        f[s] = k == 0 ? cost : k == 1 ? lx : (k < 18 ? Er[k - 2] : 0.0f);
    }
}

// Score of row l%16 (returned in every lane of that column).
__device__ __forceinline__ float mlp_tile(const MlpLane &m, const float f[5])
{
    v4f h[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 5; ++s)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(m.a1[t * 5 + s], f[s], acc, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float z = acc[v] + m.b1[t * 4 + v];
            acc[v] = z > 0.f ? z : 0.f;
        }
        h[t] = acc;
    }
    if (m.two) {
        v4f o[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 16; ++s)
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(m.a2[t * 16 + s], h[s >> 2][s & 3], acc,
                                                           0, 0, 0);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float z = acc[v] + m.b2[t * 4 + v];
                acc[v] = z > 0.f ? z : 0.f;
            }
            o[t] = acc;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) h[t] = o[t];
    }
    float part = 0.f;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) part = fmaf(m.w3[t * 4 + v], h[t][v], part);
    // sum over the four lane groups holding the same row: fixed order
    const float p16 = __shfl_xor(part, 16, WAVE);
    const float s01 = (__lane_id() & 16) ? p16 + part : part + p16; // (g0+g1) or (g2+g3)
    const float p32 = __shfl_xor(s01, 32, WAVE);
    const float tot = (__lane_id() & 32) ? p32 + s01 : s01 + p32;
    return tot + m.b3;
}

// Combine two (best, second) pairs of perturbed scores; ties go to the lower warehouse.
__device__ __forceinline__ void top2_merge(float &z1, int &w1, float &z2, float oz1, int ow1,
                                           float oz2)
{
    const bool other = oz1 > z1 || (oz1 == z1 && ow1 < w1);
    const float lose = other ? z1 : oz1;
    const float sec = other ? oz2 : z2;
    if (other) { z1 = oz1; w1 = ow1; }
    z2 = lose > sec ? lose : sec;
}

// Scores of every warehouse of one order into zbuf (perturbed, -inf without stock), by
// all waves of the workgroup: wave w takes tiles w, w + nwaves, ...
__device__ __forceinline__ void score_order(const MlpLane &m, const float *costT_r, const float *Er,
                                            const int32_t *x, int N, uint64_t seed, uint32_t traj,
                                            uint32_t t, float *zbuf, float *sbuf)
{
    const int wave = threadIdx.x / WAVE, nwaves = blockDim.x / WAVE;
    const int lane = __lane_id();
    const int ntiles = (N + 15) >> 4;
    for (int tile = wave; tile < ntiles; tile += nwaves) {
        const int w = tile * 16 + (lane & 15);
        const bool valid = w < N;
        const int xv = valid ? x[w] : 0;
        float f[5];
        lane_features(f, valid ? costT_r[w] : 0.f, log1pf((float)xv), Er);
        const float s = mlp_tile(m, f);
        if (lane < 16 && valid) {
            const float z = xv > 0 ? s + gumbel(seed, traj, t, (uint32_t)w) : -INFINITY;
            zbuf[w] = z;
            if (sbuf) sbuf[w] = s;
        }
    }
}

// Argmax (with runner-up) over zbuf[0..N) by one wave.  Returns the warehouse or LOST.
__device__ __forceinline__ int argmax_top2(const float *zbuf, int N, float &z1, float &z2)
{
    const int lane = __lane_id();
    float b1 = -INFINITY, b2 = -INFINITY;
    int w1 = 0x7fffffff;
    for (int w = lane; w < N; w += WAVE) top2_merge(b1, w1, b2, zbuf[w], w, -INFINITY);
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        const float o1 = __shfl_xor(b1, d, WAVE);
        const int ow = __shfl_xor(w1, d, WAVE);
        const float o2 = __shfl_xor(b2, d, WAVE);
        top2_merge(b1, w1, b2, o1, ow, o2);
    }
    z1 = b1;
    z2 = b2;
    return b1 == -INFINITY ? LOST : w1;
}

__device__ __forceinline__ bool near_tie(float z1, float z2)
{
    if (z2 == -INFINITY) return false;
    const float a = fabsf(z1) > fabsf(z2) ? fabsf(z1) : fabsf(z2);
    return (z1 - z2) <= 1e-5f * a;
}

// One workgroup walks one run (a process's orders of one SKU) from its entry state,
// order by order: all waves score the order's warehouses, wave 0 takes the argmax and
// applies f.  Same run bookkeeping as the greedy walk (entry state from the segmented
// scan, u of split runs, final inventory of a SKU's last run, restart frontier).
__global__ __launch_bounds__(256) void k_walk_mlp(Prob P, Plan L, const float *params, int layers,
                                                  const float *costT, int32_t *final_inv,
                                                  int has_init)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = P.N, R = P.R;
    int32_t *x = (int32_t *)smem;
    int32_t *cons = x + N;
    float *zbuf = (float *)(cons + N);
    int32_t *flag = (int32_t *)(zbuf + N); // [0] changed, [1] near ties
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    Ctl *ctl = L.ctl;
    if (ctl->done) return;
    MlpLane m;
    load_mlp(m, params, R, layers);
    const int pass = ctl->pass;
    const int32_t *fprev = L.fr[(pass - 1) & 1];
    int32_t *fcur = L.fr[pass & 1];
    const bool first = pass == 1;
    const bool all = first || L.no_frontier;
    const int n_items = all ? ctl->n_sr : ctl->n_split;
    const bool need_E = !first || has_init;
    unsigned long long n_orders = 0, n_runs = 0, n_changed = 0, n_bytes = 0, n_ties = 0;
    for (int item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int s = all ? item : L.split_list[item];
        const int g = L.sr_seg[s];
        const int s0 = L.seg_sr0[g];
        const int j = s - s0;
        if (!all) {
            const int32_t f = fprev[g];
            if (f == FR_NONE || j <= f) continue;
        }
        const int nsr = L.seg_sr0[g + 1] - s0;
        const int lo = L.sr_lo[s], hi = L.sr_lo[s + 1];
        const int key = L.seg_key[g];
        const int b = key / P.K;
        const int32_t *x0row = P.x0 + (int64_t)key * N;
        const int uidx = L.sr_uidx[s];
        const int32_t *Erow = (need_E && j > 0) ? L.E + (int64_t)uidx * N : nullptr;
        for (int w = threadIdx.x; w < N; w += blockDim.x) {
            const int32_t v = x0row[w] - (Erow ? Erow[w] : 0);
            x[w] = v > 0 ? v : 0;
            cons[w] = 0;
        }
        if (threadIdx.x == 0) { flag[0] = 0; flag[1] = 0; }
        __syncthreads();
        for (int p = lo; p < hi; ++p) {
            const int r = L.s_region[p];
            const uint32_t t = (uint32_t)L.s_t[p];
            score_order(m, costT + ((int64_t)b * R + r) * N, m.E + (int64_t)r * 16, x, N, P.seed,
                        (uint32_t)b, t, zbuf, nullptr);
            __syncthreads();
            if (wave == 0) {
                float z1, z2;
                const int a = argmax_top2(zbuf, N, z1, z2);
                if (lane == 0) {
                    const int q = L.s_qty[p];
                    int sh = 0;
                    if (a >= 0) {
                        sh = q < x[a] ? q : x[a];
                        x[a] -= sh;
                        cons[a] += q;
                    }
                    if (L.s_alpha[p] != a) { flag[0] += 1; }
                    if (near_tie(z1, z2)) flag[1] += 1;
                    L.s_alpha[p] = a;
                    L.s_ship[p] = sh;
                }
            }
            __syncthreads();
        }
        int wr = 0;
        if (uidx >= 0) {
            for (int w = threadIdx.x; w < N; w += blockDim.x) L.u[(int64_t)uidx * N + w] = cons[w];
            ++wr;
        }
        if (final_inv && j == nsr - 1) {
            for (int w = threadIdx.x; w < N; w += blockDim.x) final_inv[(int64_t)key * N + w] = x[w];
            ++wr;
        }
        if (threadIdx.x == 0) {
            const int nchg = flag[0];
            if (nchg) {
                atomicMin(&fcur[g], j);
                if (L.traj_lcp[b] < pass) atomicMax(&L.traj_lcp[b], pass);
                if (!ctl->any_changed) ctl->any_changed = 1;
            }
            n_changed += nchg;
            n_ties += flag[1];
            n_orders += hi - lo;
            n_runs += 1;
            n_bytes += 24ull * (hi - lo) + 4ull * N * (1 + (Erow ? 1 : 0) + wr);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && n_runs) {
        unsigned long long *st = ctl->stat[blockIdx.x % STAT_SLOTS];
        atomicAdd(&st[ST_ORDERS], n_orders);
        atomicAdd(&st[ST_RUNS], n_runs);
        atomicAdd(&st[ST_CHANGED], n_changed);
        atomicAdd(&st[ST_BYTES], n_bytes);
        atomicAdd(&st[ST_NEAR_TIES], n_ties);
    }
}

// Serial sweep: one workgroup per trajectory walks its orders in time order with the
// trajectory's stock in `state` ([K][N], initialised to x0); per order the SKU's stock
// row is read into LDS, scored by the same scorer, and the chosen warehouse's stock is
// written back.
__global__ __launch_bounds__(256) void k_serial_mlp(Prob P, const float *params, int layers,
                                                   const float *costT, int32_t *state,
                                                   int32_t *actions, int32_t *shipped)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = P.N, R = P.R;
    int32_t *x = (int32_t *)smem;
    float *zbuf = (float *)(x + N);
    const int b = blockIdx.x;
    if (b >= P.n_traj) return;
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    MlpLane m;
    load_mlp(m, params, R, layers);
    const int64_t t0 = P.traj_off[b], t1 = P.traj_off[b + 1];
    int32_t *xs = state + (int64_t)b * P.K * N;
    for (int64_t t = t0; t < t1; ++t) {
        int k = P.sku[t], r = P.region[t], q = P.qty[t];
        k = k < 0 ? 0 : (k >= P.K ? P.K - 1 : k); // out-of-range input never indexes memory
        r = r < 0 ? 0 : (r >= P.R ? P.R - 1 : r);
        q = q < 1 ? 1 : q;
        int32_t *xk = xs + (int64_t)k * N;
        for (int w = threadIdx.x; w < N; w += blockDim.x) x[w] = xk[w];
        __syncthreads();
        score_order(m, costT + ((int64_t)b * R + r) * N, m.E + (int64_t)r * 16, x, N, P.seed,
                    (uint32_t)b, (uint32_t)(t - t0), zbuf, nullptr);
        __syncthreads();
        if (wave == 0) {
            float z1, z2;
            const int a = argmax_top2(zbuf, N, z1, z2);
            if (lane == 0) {
                int sh = 0;
                if (a >= 0) {
                    sh = q < x[a] ? q : x[a];
                    xk[a] = x[a] - sh;
                }
                actions[t] = a;
                if (shipped) shipped[t] = sh;
            }
        }
        __threadfence_block();
        __syncthreads();
    }
}

// Diagnostic: raw scores s_w (no noise) of every warehouse for region r of trajectory b at
// inventory row xrow; one workgroup.
__global__ __launch_bounds__(256) void k_scores(Prob P, const float *params, int layers,
                                                const float *costT, int b, int r,
                                                const int32_t *xrow, float *out)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = P.N;
    int32_t *x = (int32_t *)smem;
    float *zbuf = (float *)(x + N);
    float *sbuf = zbuf + N;
    MlpLane m;
    load_mlp(m, params, P.R, layers);
    for (int w = threadIdx.x; w < N; w += blockDim.x) x[w] = xrow[w];
    __syncthreads();
    score_order(m, costT + ((int64_t)b * P.R + r) * N, m.E + (int64_t)r * 16, x, N, P.seed,
                (uint32_t)b, 0u, zbuf, sbuf);
    __syncthreads();
    for (int w = threadIdx.x; w < N; w += blockDim.x) out[w] = sbuf[w];
}

// costT[b][r][w] = (float)cost[b][w][r]: each order's cost row contiguous.
__global__ void k_cost_t(Prob P, float *costT)
{
    const int64_t n = (int64_t)P.n_traj * P.R * P.N;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int w = (int)(i % P.N);
        const int64_t br = i / P.N;
        const int r = (int)(br % P.R);
        const int64_t b = br / P.R;
        costT[i] = (float)P.cost[(b * P.N + w) * P.R + r];
    }
}

} // namespace

size_t costT_bytes(int N, int R, int n_traj) { return (size_t)n_traj * R * N * sizeof(float); }

hipError_t setup_costT(const Prob &P, float *costT, hipStream_t st)
{
    const int64_t n = (int64_t)P.n_traj * P.R * P.N;
    int64_t g = (n + 255) / 256;
    g = g < 1 ? 1 : (g > 8192 ? 8192 : g);
    hipLaunchKernelGGL(k_cost_t, dim3((unsigned)g), dim3(256), 0, st, P, costT);
    return hipGetLastError();
}

size_t walk_mlp_lds(int N) { return (size_t)N * 12 + 64; }

hipError_t launch_walk_mlp(const Prob &P, const Plan &L, const float *params, int layers,
                           const float *costT, int32_t *final_inv, bool has_init, int grid,
                           hipStream_t st)
{
    hipLaunchKernelGGL(k_walk_mlp, dim3(grid), dim3(256), walk_mlp_lds(P.N), st, P, L, params,
                       layers, costT, final_inv, has_init ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_serial_mlp(const Prob &P, const float *params, int layers, const float *costT,
                             int32_t *state, int32_t *actions, int32_t *shipped, hipStream_t st)
{
    hipLaunchKernelGGL(k_serial_mlp, dim3(P.n_traj), dim3(256), (size_t)P.N * 8 + 64, st, P,
                       params, layers, costT, state, actions, shipped);
    return hipGetLastError();
}

hipError_t launch_scores(const Prob &P, const float *params, int layers, const float *costT,
                         int b, int r, const int32_t *xrow, float *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_scores, dim3(1), dim3(256), (size_t)P.N * 12 + 64, st, P, params, layers,
                       costT, b, r, xrow, out);
    return hipGetLastError();
}

} // namespace pk

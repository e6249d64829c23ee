// Device code of the learned policy shared by the simulation and gradient kernels:
// Philox4x32-10 and the Gumbel noise, the MFMA scorers (the gradient's, with layer 1 on
// MFMA, and the simulation's, with layer 1 split by feature), argmax with runner-up.
#pragma once

#include <math.h>

#include "pk_internal.h"

namespace pk {
namespace mlpdev {

// The stock feature log(1 + x) of an integer stock x >= 0.  1 + x is exact in FP32 below
// 2^24, where log(1 + x) is well conditioned (x = 0 gives 0; x >= 1 leaves no small
// argument for log1p to protect), so logf costs a fraction of log1pf at the same accuracy.
__device__ __forceinline__ float log1p_stock(int32_t x) { return logf(1.f + (float)x); }

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
// W2 in LDS by output unit, rows W2S floats apart: the layer-2 A operands of a lane are
// four consecutive floats, and the 16-byte loads of 8 lanes fall on distinct banks.
constexpr int W2S = 68;
__host__ __device__ inline size_t w2_lds_bytes() { return (size_t)64 * W2S * sizeof(float); }

// Copies W2 into LDS (every thread of the workgroup takes part; the caller synchronises).
__device__ __forceinline__ void stage_w2(float *W2s, const float *params, int R, int layers)
{
    if (layers != 2) return;
    const float *W2 = params + (int64_t)R * 16 + 64 * 18 + 64;
    for (int i = threadIdx.x; i < 64 * 64; i += blockDim.x) W2s[(i >> 6) * W2S + (i & 63)] = W2[i];
}

struct MlpLane {
    float a1[20]; // layer 1 A operands, index t*5 + s
    float b1[16], b2[16], w3[16]; // index t*4 + v (hidden 16t + 4g + v)
    float b3;
    const float *E;   // [R][16] in global memory
    const float *W2s; // W2 in LDS (stage_w2)
    int two;          // two hidden layers
};

__device__ __forceinline__ void load_mlp(MlpLane &m, const float *params, int R, int layers,
                                         const float *W2s)
{
    const int l = __lane_id(), i = l & 15, g = l >> 4;
    const float *E = params;
    const float *W1 = E + (int64_t)R * 16;
    const float *b1 = W1 + 64 * 18;
    const float *W2 = b1 + 64;
    const float *b2 = W2 + 64 * 64;
    const float *w3 = layers == 2 ? b2 + 64 : b1 + 64;
    m.E = E;
    m.W2s = W2s;
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
    (void)W2;
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

// Hidden activations of one 16-row tile: h1 = relu(W1 f + b1) and, with two layers,
// h2 = relu(W2 h1 + b2) (one layer: h2 = h1).  D layout of the 16x16 MFMA: the lane holds
// unit 16t + 4(l/16) + v of row l%16 in h[t][v].
__device__ __forceinline__ void mlp_hidden(const MlpLane &m, const float f[5], v4f h1[4], v4f h2[4])
{
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
        h1[t] = acc;
    }
    if (m.two) {
        const int i = __lane_id() & 15, g = __lane_id() >> 4;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            v4f acc = {0.f, 0.f, 0.f, 0.f};
            // step s = 4c + v takes W2[16t + i][16c + 4g + v] with h1 unit 16c + 4g + v
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const float4 wv = *(const float4 *)(m.W2s + (16 * t + i) * W2S + 16 * c + 4 * g);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wv.x, h1[c][0], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wv.y, h1[c][1], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wv.z, h1[c][2], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wv.w, h1[c][3], acc, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float z = acc[v] + m.b2[t * 4 + v];
                acc[v] = z > 0.f ? z : 0.f;
            }
            h2[t] = acc;
        }
    } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) h2[t] = h1[t];
    }
}

// Output layer of a tile: w3 . h + b3 for row l%16 (in every lane of that column).
__device__ __forceinline__ float mlp_out(const MlpLane &m, const v4f h[4])
{
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

// Score of row l%16 (returned in every lane of that column).
__device__ __forceinline__ float mlp_tile(const MlpLane &m, const float f[5])
{
    v4f h1[4], h2[4];
    mlp_hidden(m, f, h1, h2);
    return mlp_out(m, h2);
}

// ---------------------------------------------------------------- policy scorer
// The scorer of the simulation kernels (walk, serial sweep, diagnostic scores).  Layer 1
// is split by feature: W1 f + b1 = W1[:,0] cost + W1[:,1] log1p(x) + (W1[:,2:] E[r] + b1),
// and the last term depends on the order's region only, so it is tabulated per region
// once per call (region_l1, FP32, fixed order) and layer 1 costs two FMAs per hidden unit
// on the vector ALU; only the 64 x 64 layer 2 runs on MFMA, its bias as the accumulator's
// initial value.  Lane l holds hidden units 16c + 4(l/16) + v of row l%16, the B-operand
// (and D) layout of layer 2, so no data moves between the layers.
struct ScoreLane {
    const float *W2s; // W2 in LDS (stage_w2)
    const float *Vs;  // [4][64] in LDS (stage_vectors): W1[:,0], W1[:,1], b2, w3 by unit
    float b3;
    int two;          // two hidden layers
};

// Bytes of LDS stage_vectors fills.
__host__ __device__ inline size_t vec_lds_bytes() { return (size_t)4 * 64 * sizeof(float); }

// Copies the per-unit vectors of the scorer into LDS: the cost and log1p(x) columns of W1,
// b2 (zero with one hidden layer) and w3 (every thread takes part; the caller
// synchronises).
__device__ __forceinline__ void stage_vectors(float *Vs, const float *params, int R, int layers)
{
    const float *W1 = params + (int64_t)R * 16;
    const float *b1 = W1 + 64 * 18;
    const float *b2 = b1 + 64 + 64 * 64;
    const float *w3 = layers == 2 ? b2 + 64 : b1 + 64;
    for (int i = threadIdx.x; i < 4 * 64; i += blockDim.x) {
        const int k = i >> 6, u = i & 63;
        Vs[i] = k == 0 ? W1[u * 18] : k == 1 ? W1[u * 18 + 1] : k == 2 ? (layers == 2 ? b2[u] : 0.f)
                                                                        : w3[u];
    }
}

__device__ __forceinline__ void load_score_lane(ScoreLane &m, const float *params, int R,
                                                int layers, const float *W2s, const float *Vs)
{
    const float *b1 = params + (int64_t)R * 16 + 64 * 18;
    const float *w3 = layers == 2 ? b1 + 64 + 64 * 64 + 64 : b1 + 64;
    m.W2s = W2s;
    m.Vs = Vs;
    m.two = layers == 2;
    m.b3 = w3[64];
}

// The region term of the lane's units for region r: table [R][64] (region_l1).
__device__ __forceinline__ void load_region_term(float pr[16], const float *table, int r)
{
    const int g = __lane_id() >> 4;
    const float *row = table + (int64_t)r * 64 + 4 * g;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const float4 v = *(const float4 *)(row + 16 * c);
        pr[c * 4 + 0] = v.x;
        pr[c * 4 + 1] = v.y;
        pr[c * 4 + 2] = v.z;
        pr[c * 4 + 3] = v.w;
    }
}

// Score of row l%16 (returned in every lane of that column) with the row's cost and
// log1p(stock).
__device__ __forceinline__ float score_tile(const ScoreLane &m, const float pr[16], float cost,
                                            float lx)
{
    const int i = __lane_id() & 15, g = __lane_id() >> 4;
    v4f h1[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const float4 wc = *(const float4 *)(m.Vs + 16 * c + 4 * g);
        const float4 wl = *(const float4 *)(m.Vs + 64 + 16 * c + 4 * g);
        const float a[4] = {wc.x, wc.y, wc.z, wc.w}, b[4] = {wl.x, wl.y, wl.z, wl.w};
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float z = fmaf(b[v], lx, fmaf(a[v], cost, pr[c * 4 + v]));
            h1[c][v] = z > 0.f ? z : 0.f;
        }
    }
    v4f h2[4];
    if (m.two) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const float4 bb = *(const float4 *)(m.Vs + 128 + 16 * t + 4 * g);
            v4f acc = {bb.x, bb.y, bb.z, bb.w};
            // step s = 4c + v takes W2[16t + i][16c + 4g + v] with h1 unit 16c + 4g + v
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const float4 wv = *(const float4 *)(m.W2s + (16 * t + i) * W2S + 16 * c + 4 * g);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wv.x, h1[c][0], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wv.y, h1[c][1], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wv.z, h1[c][2], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wv.w, h1[c][3], acc, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[v] = acc[v] > 0.f ? acc[v] : 0.f;
            h2[t] = acc;
        }
    } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) h2[t] = h1[t];
    }
    float part = 0.f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const float4 w = *(const float4 *)(m.Vs + 192 + 16 * t + 4 * g);
        part = fmaf(w.x, h2[t][0], part);
        part = fmaf(w.y, h2[t][1], part);
        part = fmaf(w.z, h2[t][2], part);
        part = fmaf(w.w, h2[t][3], part);
    }
    // sum over the four lane groups holding the same row: fixed order
    const float p16 = __shfl_xor(part, 16, WAVE);
    const float s01 = (__lane_id() & 16) ? p16 + part : part + p16; // (g0+g1) or (g2+g3)
    const float p32 = __shfl_xor(s01, 32, WAVE);
    const float tot = (__lane_id() & 32) ? p32 + s01 : s01 + p32;
    return tot + m.b3;
}

// Perturbed scores of the warehouses in the stock list sl[0..nf) into zl[i] (list order)
// by all waves of the workgroup: wave w takes tiles w, w + nwaves, ... (16 listed
// warehouses each), four at a time.  The noise of the four tiles' 64 rows is drawn first,
// one row per lane (lane l: row l%16 of the group's tile l/16), and lane l adds it to the
// score of that row, which it holds after scoring that tile.  lx (nullable): log1p of each
// warehouse's stock, kept by the caller as the stock changes (the same value the row
// would compute from x, once per change instead of once per row).
__device__ __forceinline__ void score_rows(const ScoreLane &m, const float pr[16],
                                           const float *costT_r, const int32_t *x,
                                           const float *lx, const int32_t *sl, int nf,
                                           uint64_t seed, uint32_t traj, uint32_t t, float *zl)
{
    const int wave = threadIdx.x / WAVE, nwaves = blockDim.x / WAVE;
    const int lane = __lane_id(), grp = lane >> 4;
    const int ntiles = (nf + 15) >> 4;
    for (int tb = wave; tb < ntiles; tb += 4 * nwaves) {
        const int mi = (tb + grp * nwaves) * 16 + (lane & 15);
        const float gn = mi < nf ? gumbel(seed, traj, t, (uint32_t)sl[mi]) : 0.f;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int tile = tb + k * nwaves;
            if (tile >= ntiles) break;
            const int i = tile * 16 + (lane & 15);
            const bool valid = i < nf;
            const int w = valid ? sl[i] : 0;
            float lv;
            if (lx) {
                lv = valid ? lx[w] : 0.f;
            } else {
                const int xv = valid ? x[w] : 0;
                lv = log1p_stock(xv);
            }
            const float s = score_tile(m, pr, valid ? costT_r[w] : 0.f, lv);
            if (grp == k && valid) zl[i] = s + gn;
        }
    }
}

// Noise-free scores of every warehouse (diagnostic), into sbuf[w], by all waves.
__device__ __forceinline__ void score_all(const ScoreLane &m, const float pr[16],
                                          const float *costT_r, const int32_t *x, int N,
                                          float *sbuf)
{
    const int wave = threadIdx.x / WAVE, nwaves = blockDim.x / WAVE;
    const int lane = __lane_id();
    for (int tile = wave; tile < (N + 15) >> 4; tile += nwaves) {
        const int w = tile * 16 + (lane & 15);
        const bool valid = w < N;
        const int xv = valid ? x[w] : 0;
        const float s = score_tile(m, pr, valid ? costT_r[w] : 0.f, log1p_stock(xv));
        if (lane < 16 && valid) sbuf[w] = s;
    }
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

// Scores of every warehouse of one order into zbuf (perturbed unless noise is false; -inf
// without stock), by all waves of the workgroup: wave w takes tiles w, w + nwaves, ...
__device__ __forceinline__ void score_order(const MlpLane &m, const float *costT_r, const float *Er,
                                            const int32_t *x, int N, uint64_t seed, uint32_t traj,
                                            uint32_t t, float *zbuf, float *sbuf, bool noise = true)
{
    const int wave = threadIdx.x / WAVE, nwaves = blockDim.x / WAVE;
    const int lane = __lane_id();
    const int ntiles = (N + 15) >> 4;
    for (int tile = wave; tile < ntiles; tile += nwaves) {
        const int w = tile * 16 + (lane & 15);
        const bool valid = w < N;
        const int xv = valid ? x[w] : 0;
        float f[5];
        lane_features(f, valid ? costT_r[w] : 0.f, log1p_stock(xv), Er);
        const float s = mlp_tile(m, f);
        if (lane < 16 && valid) {
            const float z = xv > 0 ? (noise ? s + gumbel(seed, traj, t, (uint32_t)w) : s) : -INFINITY;
            zbuf[w] = z;
            if (sbuf) sbuf[w] = s;
        }
    }
}

// Perturbed scores of the warehouses in the stock list sl[0..nf) into zbuf[w] (or, with
// by_list, into zbuf[i] for list entry i), by all waves of the workgroup (tiles of 16
// listed warehouses: wave w takes tiles w, w + nwaves, ...).  Warehouses without stock
// are not scored.
__device__ __forceinline__ void score_list(const MlpLane &m, const float *costT_r, const float *Er,
                                           const int32_t *x, const int32_t *sl, int nf,
                                           uint64_t seed, uint32_t traj, uint32_t t, float *zbuf,
                                           int first = -1, int step = 0, bool by_list = false)
{
    // by default the workgroup's waves share the tiles; first = 0, step = 1: one wave
    if (first < 0) {
        first = threadIdx.x / WAVE;
        step = blockDim.x / WAVE;
    }
    const int lane = __lane_id();
    const int ntiles = (nf + 15) >> 4;
    for (int tile = first; tile < ntiles; tile += step) {
        const int i = tile * 16 + (lane & 15);
        const bool valid = i < nf;
        const int w = valid ? sl[i] : 0;
        const int xv = valid ? x[w] : 0;
        float f[5];
        lane_features(f, valid ? costT_r[w] : 0.f, log1p_stock(xv), Er);
        const float s = mlp_tile(m, f);
        if (lane < 16 && valid) zbuf[by_list ? i : w] = s + gumbel(seed, traj, t, (uint32_t)w);
    }
}

// Top two of the (best, its warehouse, second) triples of the 64 lanes of a wave, by DPP:
// the row totals (row_shr 1, 2, 4, 8), then rows 0-1 and 2-3 (row_bcast 15), then all four
// (row_bcast 31) in lane 63, read from there.  Lanes a step does not reach keep the
// identity (-inf, no warehouse).  Merging triples of disjoint sets gives the top two of
// their union whatever the grouping, so the result equals a sequential scan's.
__device__ __forceinline__ void wave_top2(float &b1, int &w1, float &b2)
{
    const int NEG = __float_as_int(-INFINITY);
#define PK_TOP2_DPP(ctrl, rmask)                                                                 \
    {                                                                                            \
        const float o1 = __int_as_float(__builtin_amdgcn_update_dpp(NEG, __float_as_int(b1), ctrl, \
                                                                    rmask, 0xf, false));         \
        const int ow = __builtin_amdgcn_update_dpp(0x7fffffff, w1, ctrl, rmask, 0xf, false);     \
        const float o2 = __int_as_float(__builtin_amdgcn_update_dpp(NEG, __float_as_int(b2), ctrl, \
                                                                    rmask, 0xf, false));         \
        top2_merge(b1, w1, b2, o1, ow, o2);                                                      \
    }
    PK_TOP2_DPP(0x111, 0xf) // row_shr:1
    PK_TOP2_DPP(0x112, 0xf) // row_shr:2
    PK_TOP2_DPP(0x114, 0xf) // row_shr:4
    PK_TOP2_DPP(0x118, 0xf) // row_shr:8
    PK_TOP2_DPP(0x142, 0xa) // row_bcast:15 into rows 1 and 3
    PK_TOP2_DPP(0x143, 0xc) // row_bcast:31 into rows 2 and 3
#undef PK_TOP2_DPP
    b1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(b1), 63));
    w1 = __builtin_amdgcn_readlane(w1, 63);
    b2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(b2), 63));
}

// Argmax (with runner-up) of zbuf over the stock list sl[0..nf) by one wave.  Returns
// the warehouse (lowest index on exact ties) or LOST when the list is empty.
__device__ __forceinline__ int argmax_list(const float *zbuf, const int32_t *sl, int nf, float &z1,
                                           float &z2)
{
    const int lane = __lane_id();
    float b1 = -INFINITY, b2 = -INFINITY;
    int w1 = 0x7fffffff;
    for (int i = lane; i < nf; i += WAVE) {
        const int w = sl[i];
        top2_merge(b1, w1, b2, zbuf[w], w, -INFINITY);
    }
    wave_top2(b1, w1, b2);
    z1 = b1;
    z2 = b2;
    return b1 == -INFINITY ? LOST : w1;
}

// Argmax (with runner-up) of scores held in list order (zl[i] for warehouse sl[i]) by one
// wave; the score and the warehouse of an entry are independent loads.
__device__ __forceinline__ int argmax_zl(const float *zl, const int32_t *sl, int nf, float &z1,
                                         float &z2)
{
    const int lane = __lane_id();
    float b1 = -INFINITY, b2 = -INFINITY;
    int w1 = 0x7fffffff;
    for (int i = lane; i < nf; i += WAVE) top2_merge(b1, w1, b2, zl[i], sl[i], -INFINITY);
    wave_top2(b1, w1, b2);
    z1 = b1;
    z2 = b2;
    return b1 == -INFINITY ? LOST : w1;
}

// The list of warehouses with stock, x[w] > 0, in sl[0..*nf) with pos[w] its index
// there; built by wave 0 (64 warehouses per ballot).  Callers synchronise after it.
__device__ __forceinline__ void build_stock_list_wave(const int32_t *x, int N, int32_t *sl,
                                                      int32_t *pos, int32_t *nf);
__device__ __forceinline__ void build_stock_list(const int32_t *x, int N, int32_t *sl, int32_t *pos,
                                                 int32_t *nf)
{
    if (threadIdx.x < WAVE) build_stock_list_wave(x, N, sl, pos, nf);
}
// The same, by the calling wave.
__device__ __forceinline__ void build_stock_list_wave(const int32_t *x, int N, int32_t *sl,
                                                      int32_t *pos, int32_t *nf)
{
    const int lane = __lane_id();
    int base = 0;
    for (int c = 0; c < N; c += WAVE) {
        const int w = c + lane;
        const bool in = w < N && x[w] > 0;
        const uint64_t m = __ballot(in);
        if (in) {
            const int i = base + __popcll(m & lanemask_lt());
            sl[i] = w;
            pos[w] = i;
        }
        base += __popcll(m);
    }
    if (lane == 0) *nf = base;
}

// Warehouse a has just emptied: drop it from the list (the last entry takes its place).
__device__ __forceinline__ void drop_from_list(int a, int32_t *sl, int32_t *pos, int32_t *nf)
{
    const int i = pos[a];
    const int last = sl[*nf - 1];
    sl[i] = last;
    pos[last] = i;
    *nf -= 1;
}

// Algorithmic FLOPs of one scored row: 2 (18 * 64 + 64 * 64 + 64) with two hidden layers,
// 2 (18 * 64 + 64) with one.
__host__ __device__ inline unsigned long long row_flops(int layers)
{
    return layers == 2 ? 2ull * (18 * 64 + 64 * 64 + 64) : 2ull * (18 * 64 + 64);
}

// Argmax (with runner-up) over zbuf[0..N) by one wave.  Returns the warehouse or LOST.
__device__ __forceinline__ int argmax_top2(const float *zbuf, int N, float &z1, float &z2)
{
    const int lane = __lane_id();
    float b1 = -INFINITY, b2 = -INFINITY;
    int w1 = 0x7fffffff;
    for (int w = lane; w < N; w += WAVE) top2_merge(b1, w1, b2, zbuf[w], w, -INFINITY);
    wave_top2(b1, w1, b2);
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

} // namespace mlpdev
} // namespace pk

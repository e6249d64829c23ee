// REINFORCE gradient of the learned policy at fixed actions.
//
// Objective (policy gradient, Section 4.2): L = sum_t A_t log pi(a_t | s_t) with
// pi(. | s) = softmax over warehouses with stock of the scores s_w, the states s_t those
// the fixed actions induce, A_t the caller's advantages.  With p = softmax(s):
//   dL/ds_w = A_t (1[w = a_t] - p_w)   for warehouses with stock, 0 otherwise,
// back-propagated through the MLP row of each (order, warehouse) pair.  Steps with at
// most one warehouse in stock contribute nothing (log pi = 0).
//
// States: with the actions fixed, a run's entry state is x0 - E (the segmented scan of
// the runs' consumption, as in the Picard passes) and the run is walked applying the
// fixed actions.  One workgroup of four waves per run, order by order, over the list of
// warehouses with stock (rows):
//   1. the waves score the rows with the MFMA scorer (no noise); wave 0 forms the softmax
//      statistics and log pi(a_t);
//   2. the rows are taken 64 at a time, one 16-row tile per wave.  A wave recomputes its
//      tile's activations (D layout: lane holds unit 16t + 4(l/16) + v of row l%16), forms
//      the layer-2 deltas dl = ds w3 [h2 > 0] and the layer-1 deltas d1 = [h1 > 0] W2^T dl
//      (MFMA, W2^T from LDS), and keeps per-lane sums of the row-summed gradients (b1,
//      b2, w3, the cost and log1p(x) columns of W1);
//   3. h1 and dl of the 64 rows are stored by unit in LDS, so that dW2 = sum over rows of
//      dl h1^T is an MFMA product over the rows; each wave owns 16 output units of dW2;
//   4. per order the FP32 sums go into FP64 accumulators held by the lanes (each value
//      owned by one lane of one wave); the order's d1 summed over its rows gives the
//      embedding columns of dW1 (outer product with E[r]) and dE[r] (W1's embedding
//      columns times it), the latter into a per-workgroup FP64 table in global memory.
// At the end every wave writes its FP64 partial sums as one record and a final kernel sums
// the records in a fixed order: the gradient is reproducible bit for bit.
#include "mlp_device.h"

namespace pk {

namespace {

using namespace mlpdev;

constexpr int H = 64;
constexpr int GW = 4;  // waves per workgroup
constexpr int RS = 68; // LDS row stride (floats) of the by-unit tensors: 16 rows of a
                       // half wave's D-layout stores start 16 banks apart

__host__ __device__ inline int acc_count(int layers) // W1 b1 (W2 b2) w3 b3
{
    return H * 18 + H + (layers == 2 ? H * H + H : 0) + H + 1;
}

// Sums over the 16 lanes of each lane group (l/16) of 16 values per lane, scattered: lane
// m = l%16 gets the total of value m.  Butterfly with fixed pairings.
__device__ __forceinline__ float reduce_scatter16(const float v[16])
{
    const int m = __lane_id() & 15;
    const bool b8 = m & 8, b4 = m & 4, b2 = m & 2, b1 = m & 1;
    float a8[8], a4[4], a2[2];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float keep = b8 ? v[k + 8] : v[k], send = b8 ? v[k] : v[k + 8];
        a8[k] = keep + __shfl_xor(send, 8, WAVE);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float keep = b4 ? a8[k + 4] : a8[k], send = b4 ? a8[k] : a8[k + 4];
        a4[k] = keep + __shfl_xor(send, 4, WAVE);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const float keep = b2 ? a4[k + 2] : a4[k], send = b2 ? a4[k] : a4[k + 2];
        a2[k] = keep + __shfl_xor(send, 2, WAVE);
    }
    const float keep = b1 ? a2[1] : a2[0], send = b1 ? a2[0] : a2[1];
    return keep + __shfl_xor(send, 1, WAVE);
}

__global__ __launch_bounds__(256) void k_grad(Prob P, Plan L, const float *params, int layers,
                                              const float *costT, const float *adv,
                                              float *logp_sorted, double *part, double *dE_part)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = P.N, R = P.R;
    const int nacc = acc_count(layers);
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int m = lane & 15, g = lane >> 4;
    const bool two = layers == 2;
    float *W2s = (float *)smem;           // [64][W2S] W2 by output unit (the scorer's operands)
    float *W2T = W2s + 64 * W2S;          // [64][RS] W2 by input unit: W2T[i][o] = W2[o][i]
    float *H1T = W2T + H * RS;            // [64][RS] h1 of the chunk's 64 rows, by unit
    float *DLT = H1T + H * RS;            // [64][RS] layer-2 deltas of the chunk, by unit
    float *red = DLT + H * RS;            // [GW][64] each wave's d1 summed over its rows
    float *d1o = red + GW * H;            // [64] the order's d1 summed over all rows
    float *Ebuf = d1o + H;                // [16] embedding of the order's region
    float *misc = Ebuf + 16;              // [0] max score, [1] log Z
    int32_t *imisc = (int32_t *)(misc + 4); // [0] skip the order
    int32_t *x = imisc + 4;               // [N] stock
    float *sbuf = (float *)(x + N);       // [N] scores
    int32_t *sl = (int32_t *)(sbuf + N);  // [N] warehouses with stock
    int32_t *pos = sl + N;                // [N] their index in sl
    int32_t *nfp = pos + N;               // [1] how many
    float *lxs = (float *)(nfp + 4);      // [N] log1p of each warehouse's stock
    // parameter views
    const float *W1 = params + (int64_t)R * 16;
    const float *b1 = W1 + H * 18;
    const float *W2 = b1 + H;
    stage_w2(W2s, params, R, layers); // read after the barrier below
    MlpLane mw;
    load_mlp(mw, params, R, layers, W2s);
    if (two)
        for (int i = threadIdx.x; i < H * H; i += blockDim.x) W2T[(i % H) * RS + i / H] = W2[i];
    float w1e[16]; // W1[lane][2 + k]: the embedding columns (wave 0 forms dE with them)
#pragma unroll
    for (int k = 0; k < 16; ++k) w1e[k] = W1[lane * 18 + 2 + k];
    __syncthreads();
    // FP64 accumulators, each value owned by one lane of one wave
    double gW2[16];                       // units o = 16 wave + 4g + v, inputs i = 16T + m
#pragma unroll
    for (int k = 0; k < 16; ++k) gW2[k] = 0.0;
    double gb1 = 0.0, gb2 = 0.0, gw3 = 0.0, gc0 = 0.0, gc1 = 0.0, gb3 = 0.0, gobj = 0.0;
    double gW1E[4] = {0.0, 0.0, 0.0, 0.0}; // W1[tid / 4][2 + 4 (tid % 4) + k]
    const v4f zero4 = {0.f, 0.f, 0.f, 0.f};
    v4f aW2[4] = {zero4, zero4, zero4, zero4}; // this order's dW2 share (FP32)
    double *dEw = dE_part + (int64_t)blockIdx.x * R * 16;
    const int n_items = L.ctl->n_sr;
    for (int item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int s = item;
        const int gseg = L.sr_seg[s];
        const int jr = s - L.seg_sr0[gseg];
        const int lo = L.sr_lo[s], hi = L.sr_lo[s + 1];
        const int key = L.seg_key[gseg];
        const int b = key / P.K;
        const int32_t *x0row = P.x0 + (int64_t)key * N;
        const int uidx = L.sr_uidx[s];
        const int32_t *Erow = jr > 0 ? L.E + (int64_t)uidx * N : nullptr;
        for (int w = threadIdx.x; w < N; w += blockDim.x) {
            const int32_t v = x0row[w] - (Erow ? Erow[w] : 0);
            x[w] = v > 0 ? v : 0;
            lxs[w] = log1p_stock(v > 0 ? v : 0);
        }
        __syncthreads();
        build_stock_list(x, N, sl, pos, nfp);
        __syncthreads();
        for (int p = lo; p < hi; ++p) {
            const int r = L.s_region[p];
            const int a = L.s_alpha[p];
            const float A = adv[L.perm[p]];
            const float *cr = costT + ((int64_t)b * R + r) * N;
            if (threadIdx.x < 16) Ebuf[threadIdx.x] = mw.E[(int64_t)r * 16 + threadIdx.x];
            __syncthreads();
            const int nf = *nfp;
            // 1. scores of the rows
            const int ntiles = (nf + 15) >> 4;
            for (int tile = wave; tile < ntiles; tile += GW) {
                const int i = tile * 16 + m;
                const bool valid = i < nf;
                const int w = valid ? sl[i] : 0;
                float f[5];
                lane_features(f, valid ? cr[w] : 0.f, valid ? lxs[w] : 0.f, Ebuf);
                const float sc = mlp_tile(mw, f);
                if (lane < 16 && valid) sbuf[w] = sc;
            }
            __syncthreads();
            if (wave == 0) {
                float mx = -INFINITY;
                for (int i = lane; i < nf; i += WAVE) mx = fmaxf(mx, sbuf[sl[i]]);
#pragma unroll
                for (int d = 32; d > 0; d >>= 1) mx = fmaxf(mx, __shfl_xor(mx, d, WAVE));
                float se = 0.f;
                for (int i = lane; i < nf; i += WAVE) se += expf(sbuf[sl[i]] - mx);
#pragma unroll
                for (int d = 32; d > 0; d >>= 1) se += __shfl_xor(se, d, WAVE);
                if (lane == 0) {
                    const bool bad = a >= 0 ? (a >= N || x[a] <= 0) : nf > 0;
                    if (bad) atomicOr(&L.ctl->error, 8);
                    float lp = 0.f;
                    if (!bad && nf > 1) lp = sbuf[a] - (mx + logf(se));
                    logp_sorted[p] = lp;
                    gobj += (double)A * (double)lp;
                    misc[0] = mx;
                    misc[1] = logf(se);
                    imisc[0] = bad || nf <= 1 || A == 0.f;
                }
            }
            __syncthreads();
            if (!imisc[0]) {
                const float mx = misc[0], lz = misc[1];
                float pb1[16], pb2[16], pw3[16], pc0[16], pc1[16], pb3 = 0.f;
#pragma unroll
                for (int k = 0; k < 16; ++k) pb1[k] = pb2[k] = pw3[k] = pc0[k] = pc1[k] = 0.f;
                for (int c0 = 0; c0 < nf; c0 += 64) {
                    const int row0 = c0 + 16 * wave; // this wave's tile of the chunk
                    if (row0 < nf) {
                        // 2. activations and deltas of the tile
                        const int i = row0 + m;
                        const bool valid = i < nf;
                        const int w = valid ? sl[i] : 0;
                        const float cost = valid ? cr[w] : 0.f, lx = valid ? lxs[w] : 0.f;
                        float f[5];
                        lane_features(f, cost, lx, Ebuf);
                        v4f h1[4], h2[4], d1[4];
                        mlp_hidden(mw, f, h1, h2);
                        const float ds =
                            valid ? A * ((w == a ? 1.f : 0.f) - expf(sbuf[w] - mx - lz)) : 0.f;
                        if (g == 0) pb3 += ds;
                        if (two) {
                            v4f dl[4];
#pragma unroll
                            for (int t = 0; t < 4; ++t)
#pragma unroll
                                for (int v = 0; v < 4; ++v) {
                                    dl[t][v] = h2[t][v] > 0.f ? ds * mw.w3[t * 4 + v] : 0.f;
                                    pw3[t * 4 + v] = fmaf(ds, h2[t][v], pw3[t * 4 + v]);
                                    pb2[t * 4 + v] += dl[t][v];
                                }
                            // d1 = [h1 > 0] W2^T dl: A = W2^T (unit i = 16T + m, chunk units
                            // o = 16t + 4g + v), B = dl in its D layout
#pragma unroll
                            for (int T = 0; T < 4; ++T) {
                                v4f acc = zero4;
#pragma unroll
                                for (int t = 0; t < 4; ++t) {
                                    const float4 wv =
                                        *(const float4 *)(W2T + (16 * T + m) * RS + 16 * t + 4 * g);
                                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wv.x, dl[t][0], acc, 0, 0, 0);
                                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wv.y, dl[t][1], acc, 0, 0, 0);
                                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wv.z, dl[t][2], acc, 0, 0, 0);
                                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wv.w, dl[t][3], acc, 0, 0, 0);
                                }
#pragma unroll
                                for (int v = 0; v < 4; ++v) d1[T][v] = h1[T][v] > 0.f ? acc[v] : 0.f;
                            }
                            // 3. the tile's rows of h1 and dl, by unit
#pragma unroll
                            for (int t = 0; t < 4; ++t)
#pragma unroll
                                for (int v = 0; v < 4; ++v) {
                                    const int at = (16 * t + 4 * g + v) * RS + 16 * wave + m;
                                    H1T[at] = h1[t][v];
                                    DLT[at] = dl[t][v];
                                }
                        } else {
#pragma unroll
                            for (int t = 0; t < 4; ++t)
#pragma unroll
                                for (int v = 0; v < 4; ++v) {
                                    d1[t][v] = h1[t][v] > 0.f ? ds * mw.w3[t * 4 + v] : 0.f;
                                    pw3[t * 4 + v] = fmaf(ds, h1[t][v], pw3[t * 4 + v]);
                                }
                        }
#pragma unroll
                        for (int t = 0; t < 4; ++t)
#pragma unroll
                            for (int v = 0; v < 4; ++v) {
                                pb1[t * 4 + v] += d1[t][v];
                                pc0[t * 4 + v] = fmaf(d1[t][v], cost, pc0[t * 4 + v]);
                                pc1[t * 4 + v] = fmaf(d1[t][v], lx, pc1[t * 4 + v]);
                            }
                    } else if (two) { // no rows: zero deltas (and finite activations)
#pragma unroll
                        for (int t = 0; t < 4; ++t)
#pragma unroll
                            for (int v = 0; v < 4; ++v) {
                                const int at = (16 * t + 4 * g + v) * RS + 16 * wave + m;
                                H1T[at] = 0.f;
                                DLT[at] = 0.f;
                            }
                    }
                    if (two) {
                        __syncthreads();
                        // dW2[o][i] += sum over the chunk's rows of dl[o] h1[i]: this wave's
                        // units o = 16 wave + ..; rows 16g + c (c < 16) are lane group g's
                        const float4 *ap = (const float4 *)(DLT + (16 * wave + m) * RS + 16 * g);
                        const float4 a0 = ap[0], a1 = ap[1], a2 = ap[2], a3 = ap[3];
                        const float av[16] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w,
                                              a2.x, a2.y, a2.z, a2.w, a3.x, a3.y, a3.z, a3.w};
#pragma unroll
                        for (int T = 0; T < 4; ++T) {
                            const float4 *bp = (const float4 *)(H1T + (16 * T + m) * RS + 16 * g);
                            const float4 q0 = bp[0], q1 = bp[1], q2 = bp[2], q3 = bp[3];
                            const float bv[16] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w,
                                                  q2.x, q2.y, q2.z, q2.w, q3.x, q3.y, q3.z, q3.w};
#pragma unroll
                            for (int c = 0; c < 16; ++c)
                                aW2[T] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[c], bv[c], aW2[T], 0, 0, 0);
                        }
                        __syncthreads();
                    }
                }
                // 4. the order's sums into FP64
                if (two) {
#pragma unroll
                    for (int T = 0; T < 4; ++T) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) gW2[T * 4 + v] += (double)aW2[T][v];
                        aW2[T] = zero4;
                    }
                    gb2 += (double)reduce_scatter16(pb2);
                }
                const float rb1 = reduce_scatter16(pb1);
                gb1 += (double)rb1;
                gw3 += (double)reduce_scatter16(pw3);
                gc0 += (double)reduce_scatter16(pc0);
                gc1 += (double)reduce_scatter16(pc1);
                gb3 += (double)pb3;
                red[wave * H + 16 * (m >> 2) + 4 * g + (m & 3)] = rb1;
                __syncthreads();
                if (threadIdx.x < H)
                    d1o[threadIdx.x] = ((red[threadIdx.x] + red[H + threadIdx.x]) +
                                        red[2 * H + threadIdx.x]) + red[3 * H + threadIdx.x];
                __syncthreads();
                {
                    const double d = (double)d1o[threadIdx.x >> 2];
                    const int k0 = 4 * (threadIdx.x & 3);
#pragma unroll
                    for (int k = 0; k < 4; ++k) gW1E[k] += (double)Ebuf[k0 + k] * d;
                }
                if (wave == 0) { // dE[r][k] += sum_j W1[j][2 + k] d1o[j]
                    const float d = d1o[lane];
                    float v[16];
#pragma unroll
                    for (int k = 0; k < 16; ++k) v[k] = w1e[k] * d;
                    float t = reduce_scatter16(v);
                    t = t + __shfl_xor(t, 16, WAVE);
                    t = t + __shfl_xor(t, 32, WAVE);
                    if (lane < 16) dEw[(int64_t)r * 16 + lane] += (double)t;
                }
            }
            __syncthreads();
            if (threadIdx.x == 0 && a >= 0 && a < N) { // the fixed action
                const int q = L.s_qty[p];
                const int xa = x[a];
                const int nx = xa - (q < xa ? q : xa);
                x[a] = nx;
                lxs[a] = log1p_stock(nx);
                if (xa > 0 && nx == 0) drop_from_list(a, sl, pos, nfp);
            }
            __syncthreads();
        }
    }
    // this wave's record (the records were zeroed; every value is written by its owner)
    double *rec = part + ((int64_t)blockIdx.x * GW + wave) * (nacc + 1);
    const int oW1 = 0, ob1 = H * 18, oW2 = ob1 + H, ob2 = oW2 + (two ? H * H : 0);
    const int ow3 = two ? ob2 + H : ob1 + H, ob3 = ow3 + H;
    const int u = 16 * (m >> 2) + 4 * g + (m & 3); // unit of this lane's scattered sums
    rec[ob1 + u] = gb1;
    rec[oW1 + u * 18] = gc0;
    rec[oW1 + u * 18 + 1] = gc1;
    rec[ow3 + u] = gw3;
    if (two) {
        rec[ob2 + u] = gb2;
#pragma unroll
        for (int T = 0; T < 4; ++T)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                rec[oW2 + (16 * wave + 4 * g + v) * H + 16 * T + m] = gW2[T * 4 + v];
    }
    {
        const int i = threadIdx.x >> 2, k0 = 4 * (threadIdx.x & 3);
#pragma unroll
        for (int k = 0; k < 4; ++k) rec[oW1 + i * 18 + 2 + k0 + k] = gW1E[k];
    }
    double t3 = gb3; // lanes of group 0 hold their rows' sums; butterfly in a fixed order
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) t3 += __shfl_xor(t3, d, WAVE);
    if (lane == 0) rec[ob3] = t3;
    if (wave == 0 && lane == 0) rec[nacc] = gobj;
}

__global__ void k_zero_f64(double *p, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0.0;
}

// grad[i] = sum over the records of the partials, in record order (FP64): one dE table per
// workgroup, one record per wave.
__global__ void k_grad_reduce(const double *part, const double *dE_part, int n_wg, int R,
                              int layers, float *grad, double *objective)
{
    const int nacc = acc_count(layers);
    const int nE = R * 16;
    const int n = nE + nacc;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += gridDim.x * blockDim.x) {
        double s = 0.0;
        if (i < nE)
            for (int w = 0; w < n_wg; ++w) s += dE_part[(int64_t)w * nE + i];
        else
            for (int w = 0; w < n_wg * GW; ++w) s += part[(int64_t)w * (nacc + 1) + (i - nE)];
        if (i < n) {
            if (grad) grad[i] = (float)s;
        } else {
            *objective = s;
        }
    }
}

__global__ void k_unpermute_f32(const int32_t *perm, const float *src, float *dst, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride)
        dst[perm[p]] = src[p];
}

} // namespace

size_t grad_lds(int N, int layers)
{
    (void)layers;
    return w2_lds_bytes() + (size_t)(3 * H * RS + GW * H + H + 16 + 4) * 4 + 16 + (size_t)N * 20 + 32;
}

size_t grad_part_bytes(int n_wg, int R, int layers)
{
    return (size_t)n_wg * GW * (acc_count(layers) + 1) * 8 + (size_t)n_wg * R * 16 * 8;
}

hipError_t launch_grad(const Prob &P, const Plan &L, const float *params, int layers,
                       const float *costT, const float *adv, float *logp_sorted, double *part,
                       int n_wg, float *grad, double *objective_dev, float *logp_out,
                       hipStream_t st)
{
    const int64_t n_rec = (int64_t)n_wg * GW * (acc_count(layers) + 1);
    double *dE_part = part + n_rec;
    const int64_t nz = n_rec + (int64_t)n_wg * P.R * 16; // records and dE tables start at 0
    hipLaunchKernelGGL(k_zero_f64, dim3(1024), dim3(256), 0, st, part, nz);
    hipLaunchKernelGGL(k_grad, dim3(n_wg), dim3(256), grad_lds(P.N, layers), st, P, L, params,
                       layers, costT, adv, logp_sorted, part, dE_part);
    const int n = P.R * 16 + acc_count(layers) + 1;
    hipLaunchKernelGGL(k_grad_reduce, dim3((n + 255) / 256), dim3(256), 0, st, part, dE_part, n_wg,
                       P.R, layers, grad, objective_dev);
    if (logp_out) {
        int64_t g = (P.total + 255) / 256;
        g = g < 1 ? 1 : (g > 8192 ? 8192 : g);
        hipLaunchKernelGGL(k_unpermute_f32, dim3((unsigned)g), dim3(256), 0, st, L.perm,
                           logp_sorted, logp_out, P.total);
    }
    return hipGetLastError();
}

} // namespace pk

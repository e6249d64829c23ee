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
// fixed actions.  One workgroup per run, order by order:
//   1. all waves score the order's warehouses with the MFMA scorer (no noise);
//   2. wave 0 forms the softmax statistics and log pi(a_t);
//   3. the rows with stock are split over the waves; a wave recomputes one row's
//      activations with one lane per hidden unit (weights of the lane's unit in
//      registers, the row's hidden vector broadcast through LDS) and back-propagates
//      into per-lane FP32 accumulators;
//   4. per order the FP32 accumulators (at most a few hundred terms) are added into the
//      workgroup's FP64 accumulators in LDS; embedding gradients go to a per-workgroup
//      FP64 table in global memory.
// At the end each workgroup writes its FP64 partial sums and a final kernel sums them
// over workgroups in a fixed order.
#include "mlp_device.h"

namespace pk {

namespace {

using namespace mlpdev;

constexpr int H = 64;

__host__ __device__ inline int acc_count(int layers) // W1 b1 (W2 b2) w3 b3
{
    return H * 18 + H + (layers == 2 ? H * H + H : 0) + H + 1;
}

__global__ __launch_bounds__(256) void k_grad(Prob P, Plan L, const float *params, int layers,
                                              const float *costT, const float *adv,
                                              float *logp_sorted, double *part, double *dE_part)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = P.N, R = P.R;
    const int nacc = acc_count(layers);
    double *acc = (double *)smem;                  // [nacc]
    double *obj = acc + nacc;                      // [1]
    float *misc = (float *)(obj + 1);              // [0] max, [1] log Z
    int32_t *imisc = (int32_t *)(misc + 2);        // [0] n feasible, [1] action, [2] skip
    float *Ebuf = (float *)(imisc + 4);            // [16] embedding of the order's region
    float *d1sum = Ebuf + 16;                      // [64]
    float *hbuf = d1sum + H;                       // [4][64]
    float *dbuf = hbuf + 4 * H;                    // [4][64]
    float *W2s = dbuf + 4 * H;                     // [64][65] W2, rows padded (no bank conflicts
                                                   // for row or column access)
    int32_t *x = (int32_t *)(W2s + H * (H + 1));   // [N]
    float *sbuf = (float *)(x + N);                // [N]
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int two = layers == 2;
    // parameter views
    const float *E = params;
    const float *W1 = E + (int64_t)R * 16;
    const float *b1 = W1 + H * 18;
    const float *W2 = b1 + H;
    const float *b2 = W2 + H * H;
    const float *w3 = two ? b2 + H : b1 + H;
    // accumulator offsets (parameter order after the embedding)
    const int oW1 = 0, ob1 = H * 18, oW2 = ob1 + H, ob2 = oW2 + (two ? H * H : 0);
    const int ow3 = two ? ob2 + H : ob1 + H, ob3 = ow3 + H;
    // this lane's hidden unit j = lane
    const int j = lane;
    const float b1j = b1[j], b2j = two ? b2[j] : 0.f, w3j = w3[j];
    for (int i = threadIdx.x; i < nacc + 1; i += blockDim.x) acc[i] = 0.0;
    if (two)
        for (int i = threadIdx.x; i < H * H; i += blockDim.x) W2s[(i / H) * (H + 1) + i % H] = W2[i];
    for (int i = threadIdx.x; i < H; i += blockDim.x) d1sum[i] = 0.f;
    __syncthreads();
    double *dEw = dE_part + (int64_t)blockIdx.x * R * 16;
    const int n_items = L.ctl->n_sr;
    for (int item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int s = item;
        const int g = L.sr_seg[s];
        const int s0 = L.seg_sr0[g];
        const int jr = s - s0;
        const int lo = L.sr_lo[s], hi = L.sr_lo[s + 1];
        const int key = L.seg_key[g];
        const int b = key / P.K;
        const int32_t *x0row = P.x0 + (int64_t)key * N;
        const int uidx = L.sr_uidx[s];
        const int32_t *Erow = jr > 0 ? L.E + (int64_t)uidx * N : nullptr;
        for (int w = threadIdx.x; w < N; w += blockDim.x) {
            const int32_t v = x0row[w] - (Erow ? Erow[w] : 0);
            x[w] = v > 0 ? v : 0;
        }
        __syncthreads();
        for (int p = lo; p < hi; ++p) {
            const int r = L.s_region[p];
            const int a = L.s_alpha[p];
            const float A = adv[L.perm[p]];
            const float *cr = costT + ((int64_t)b * R + r) * N;
            if (threadIdx.x < 16) Ebuf[threadIdx.x] = E[(int64_t)r * 16 + threadIdx.x];
            { // scorer weights live only for this phase (they are re-read from cache)
                MlpLane m;
                load_mlp(m, params, R, layers);
                score_order(m, cr, m.E + (int64_t)r * 16, x, N, 0, 0, 0, sbuf, nullptr, false);
            }
            __syncthreads();
            if (wave == 0) {
                float mx = -INFINITY;
                int nf = 0;
                for (int w = lane; w < N; w += WAVE) {
                    const float v = sbuf[w];
                    if (v != -INFINITY) { mx = v > mx ? v : mx; ++nf; }
                }
#pragma unroll
                for (int d = 32; d > 0; d >>= 1) {
                    const float o = __shfl_xor(mx, d, WAVE);
                    mx = o > mx ? o : mx;
                    nf += __shfl_xor(nf, d, WAVE);
                }
                float se = 0.f;
                for (int w = lane; w < N; w += WAVE) {
                    const float v = sbuf[w];
                    if (v != -INFINITY) se += expf(v - mx);
                }
#pragma unroll
                for (int d = 32; d > 0; d >>= 1) se += __shfl_xor(se, d, WAVE);
                if (lane == 0) {
                    const bool bad = a >= 0 ? (a >= N || x[a] <= 0) : nf > 0;
                    if (bad) atomicOr(&L.ctl->error, 8);
                    float lp = 0.f;
                    if (!bad && nf > 1) lp = sbuf[a] - (mx + logf(se));
                    logp_sorted[p] = lp;
                    *obj += (double)A * (double)lp;
                    misc[0] = mx;
                    misc[1] = logf(se);
                    imisc[0] = nf;
                    imisc[1] = a;
                    imisc[2] = bad || nf <= 1 || A == 0.f;
                }
            }
            __syncthreads();
            if (!imisc[2]) {
                const float mx = misc[0], lz = misc[1];
                float w1[18];
#pragma unroll
                for (int k = 0; k < 18; ++k) w1[k] = W1[j * 18 + k];
                const float *w2row = W2s + j * (H + 1); // W2[j][.]
                const float *w2col = W2s + j;          // W2[.][j], stride H + 1
                float aw1[18], aw2[H];
                float ab1 = 0.f, ab2 = 0.f, aw3 = 0.f, ab3 = 0.f, d1s = 0.f;
#pragma unroll
                for (int k = 0; k < 18; ++k) aw1[k] = 0.f;
#pragma unroll
                for (int i = 0; i < H; ++i) aw2[i] = 0.f;
                float f[18];
#pragma unroll
                for (int k = 0; k < 16; ++k) f[2 + k] = Ebuf[k];
                float *hb = hbuf + wave * H, *db = dbuf + wave * H;
                for (int w = wave; w < N; w += 4) {
                    const float sw = sbuf[w];
                    if (sw == -INFINITY) continue; // wave-uniform
                    const float pw = expf(sw - mx - lz);
                    const float ds = A * ((w == a ? 1.f : 0.f) - pw);
                    f[0] = cr[w];
                    f[1] = log1pf((float)x[w]);
                    float pre1 = b1j;
#pragma unroll
                    for (int k = 0; k < 18; ++k) pre1 = fmaf(w1[k], f[k], pre1);
                    const float h1 = pre1 > 0.f ? pre1 : 0.f;
                    float hl = h1, pre2 = 0.f;
                    hb[j] = h1;
                    wave_sync();
                    if (two) {
                        pre2 = b2j;
#pragma unroll
                        for (int i = 0; i < H; ++i) pre2 = fmaf(w2row[i], hb[i], pre2);
                        hl = pre2 > 0.f ? pre2 : 0.f;
                    }
                    aw3 = fmaf(ds, hl, aw3);
                    ab3 += ds;
                    const float dl = ((two ? pre2 : pre1) > 0.f) ? ds * w3j : 0.f;
                    float d1 = dl;
                    if (two) {
                        ab2 += dl;
#pragma unroll
                        for (int i = 0; i < H; ++i) aw2[i] = fmaf(dl, hb[i], aw2[i]);
                        db[j] = dl;
                        wave_sync();
                        float t = 0.f;
#pragma unroll
                        for (int o = 0; o < H; ++o) t = fmaf(w2col[o * (H + 1)], db[o], t);
                        d1 = pre1 > 0.f ? t : 0.f;
                    }
                    ab1 += d1;
#pragma unroll
                    for (int k = 0; k < 18; ++k) aw1[k] = fmaf(d1, f[k], aw1[k]);
                    d1s += d1;
                    wave_sync();
                }
                // this order's sums into the workgroup's FP64 accumulators, one wave after
                // the other in a fixed order (the gradient is reproducible bit for bit)
                for (int wv = 0; wv < 4; ++wv) {
                    if (wave == wv) {
#pragma unroll
                        for (int k = 0; k < 18; ++k) acc[oW1 + j * 18 + k] += (double)aw1[k];
                        acc[ob1 + j] += (double)ab1;
                        if (two) {
#pragma unroll
                            for (int i = 0; i < H; ++i) acc[oW2 + j * H + i] += (double)aw2[i];
                            acc[ob2 + j] += (double)ab2;
                        }
                        acc[ow3 + j] += (double)aw3;
                        if (lane == 0) acc[ob3] += (double)ab3;
                        d1sum[j] += d1s;
                    }
                    __syncthreads();
                }
            }
            __syncthreads();
            if (wave == 0) {
                if (!imisc[2]) {
                    // dL/dE[r][k] = sum_j W1[j][2+k] * (sum over rows of d1_j)
                    const float ds1 = d1sum[j];
                    for (int k = 0; k < 16; ++k) {
                        float v = W1[j * 18 + 2 + k] * ds1;
#pragma unroll
                        for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, WAVE);
                        if (lane == k) dEw[(int64_t)r * 16 + k] += (double)v;
                    }
                    d1sum[j] = 0.f;
                }
                if (lane == 0 && a >= 0 && a < N) {
                    const int q = L.s_qty[p];
                    x[a] -= q < x[a] ? q : x[a];
                }
            }
            __syncthreads();
        }
    }
    double *pw = part + (int64_t)blockIdx.x * (nacc + 1);
    for (int i = threadIdx.x; i < nacc + 1; i += blockDim.x) pw[i] = acc[i];
}

__global__ void k_zero_f64(double *p, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0.0;
}

// grad[i] = sum over workgroups of the partials, in workgroup order (FP64).
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
            for (int w = 0; w < n_wg; ++w) s += part[(int64_t)w * (nacc + 1) + (i - nE)];
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
    return (size_t)(acc_count(layers) + 1) * 8 + 64 + 16 * 4 + H * 4 + 8 * H * 4 +
           (size_t)H * (H + 1) * 4 + (size_t)N * 8 + 64;
}

size_t grad_part_bytes(int n_wg, int R, int layers)
{
    return (size_t)n_wg * (acc_count(layers) + 1) * 8 + (size_t)n_wg * R * 16 * 8;
}

hipError_t launch_grad(const Prob &P, const Plan &L, const float *params, int layers,
                       const float *costT, const float *adv, float *logp_sorted, double *part,
                       int n_wg, float *grad, double *objective_dev, float *logp_out,
                       hipStream_t st)
{
    double *dE_part = part + (int64_t)n_wg * (acc_count(layers) + 1);
    const int64_t nE = (int64_t)n_wg * P.R * 16;
    hipLaunchKernelGGL(k_zero_f64, dim3(1024), dim3(256), 0, st, dE_part, nE);
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

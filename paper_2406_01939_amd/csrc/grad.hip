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
// warehouses with stock (rows), 16-row tiles, wave w taking tiles w, w + 4, ...:
//   1. each wave scores its tiles with the policy scorer's arithmetic (layer 1 from the
//      per-region table on the vector ALU, layer 2 on MFMA; D layout: lane holds unit
//      16t + 4(l/16) + v of row l%16) and keeps the activations of its first tile in
//      registers; a running (max, sum of exp) per lane gives the wave's softmax partials,
//      which the waves combine after one barrier;
//   2. per chunk of 64 rows (one tile per wave) a wave forms its tile's layer-2 deltas
//      dl = ds w3 [h2 > 0] and layer-1 deltas d1 = [h1 > 0] W2^T dl (MFMA, W2^T read from
//      the staged W2) and sums the row-summed gradients of the tile (b1, w3, the cost and
//      log1p(x) columns of W1) over its rows; later tiles are scored again here;
//   3. h1 and dl of the chunk's 64 rows are stored by unit in LDS, so that dW2 = sum over
//      rows of dl h1^T is an MFMA product over the rows (over the chunk's tiles only);
//      each wave owns 16 output units of dW2 (and of db2, the row sums of its dl rows);
//   4. the order's d1 summed over its rows gives the embedding columns of dW1 (outer
//      product with E[r]) and dE[r] (W1's embedding columns times it), the latter into a
//      per-workgroup FP64 table in global memory.
// Each lane sums its share of the gradient over runs of about 2048 orders in FP32 and adds
// it to its wave's FP64 record (each value owned by one lane); a final kernel sums
// the records in a fixed order: the gradient is reproducible bit for bit.
#include "mlp_device.h"

namespace pk {

namespace {

using namespace mlpdev;

constexpr int H = 64;
constexpr int GW = 4;   // waves per workgroup
constexpr int RS = 68;  // LDS row stride (floats) of the by-unit tensors: 16 rows of a
                        // half wave's D-layout stores start 16 banks apart
constexpr int W1ES = 17; // row stride of W1's embedding columns in LDS
constexpr int FLUSH = 2048; // orders between additions of the FP32 sums to the FP64 records
constexpr int KEEP = 1;  // tiles per wave whose activations stay in registers from the
                         // scores to the backward pass (later tiles are scored again)

__host__ __device__ inline int acc_count(int layers) // W1 b1 (W2 b2) w3 b3
{
    return H * 18 + H + (layers == 2 ? H * H + H : 0) + H + 1;
}

// Value of the lane that the DPP control CTRL selects (within each row of 16 lanes).
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, true));
}

// Sums over the 16 lanes of each lane group (l/16) of 16 values per lane, scattered: lane
// m = l%16 gets the total of value m.  Butterfly with fixed pairings, on DPP lane moves:
// partners m ^ 8 (row rotation by 8), m ^ 7 (half-row mirror), m ^ 2 and m ^ 1 (quad
// permutations); the decision bits 3, 2, 1, 0 of m pick which half a lane keeps, and the
// four masks span the 16 lanes, so lane m ends with value m summed over all of them.
__device__ __forceinline__ float reduce_scatter16(const float v[16])
{
    const int m = __lane_id() & 15;
    const bool b8 = m & 8, b4 = m & 4, b2 = m & 2, b1 = m & 1;
    float a8[8], a4[4], a2[2];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float keep = b8 ? v[k + 8] : v[k], send = b8 ? v[k] : v[k + 8];
        a8[k] = keep + dpp_f<0x128>(send);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float keep = b4 ? a8[k + 4] : a8[k], send = b4 ? a8[k] : a8[k + 4];
        a4[k] = keep + dpp_f<0x141>(send);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const float keep = b2 ? a4[k + 2] : a4[k], send = b2 ? a4[k] : a4[k + 2];
        a2[k] = keep + dpp_f<0x4e>(send);
    }
    const float keep = b1 ? a2[1] : a2[0], send = b1 ? a2[0] : a2[1];
    return keep + dpp_f<0xb1>(send);
}

// Activations and score of one 16-row tile (the policy scorer's arithmetic): h1, h2 in the
// D layout, the score of row l%16 returned in every lane of that column.
__device__ __forceinline__ float tile_forward(const float *W2s, const float *Vs, bool two,
                                              float b3, const float *prL, float cost, float lx,
                                              v4f h1[4], v4f h2[4])
{
    const int i = __lane_id() & 15, g = __lane_id() >> 4;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const float4 wc = *(const float4 *)(Vs + 16 * c + 4 * g);
        const float4 wl = *(const float4 *)(Vs + 64 + 16 * c + 4 * g);
        const float4 pv = *(const float4 *)(prL + 16 * c + 4 * g);
        const float a[4] = {wc.x, wc.y, wc.z, wc.w}, b[4] = {wl.x, wl.y, wl.z, wl.w};
        const float pr[4] = {pv.x, pv.y, pv.z, pv.w};
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float z = fmaf(b[v], lx, fmaf(a[v], cost, pr[v]));
            h1[c][v] = z > 0.f ? z : 0.f;
        }
    }
    if (two) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const float4 bb = *(const float4 *)(Vs + 128 + 16 * t + 4 * g);
            v4f acc = {bb.x, bb.y, bb.z, bb.w};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const float4 wv = *(const float4 *)(W2s + (16 * t + i) * W2S + 16 * c + 4 * g);
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
        const float4 w = *(const float4 *)(Vs + 192 + 16 * t + 4 * g);
        part = fmaf(w.x, h2[t][0], part);
        part = fmaf(w.y, h2[t][1], part);
        part = fmaf(w.z, h2[t][2], part);
        part = fmaf(w.w, h2[t][3], part);
    }
    const float p16 = __shfl_xor(part, 16, WAVE);
    const float s01 = (__lane_id() & 16) ? p16 + part : part + p16;
    const float p32 = __shfl_xor(s01, 32, WAVE);
    const float tot = (__lane_id() & 32) ? p32 + s01 : s01 + p32;
    return tot + b3;
}

// Running softmax partials of one lane over the rows it holds: (max, sum of exp(s - max)).
__device__ __forceinline__ void online_lse(float &mx, float &se, float s)
{
    if (s > mx) {
        se = se * expf(mx - s) + 1.f;
        mx = s;
    } else {
        se += expf(s - mx);
    }
}

__global__ __launch_bounds__(256, 2) void k_grad(Prob P, Plan L, const float *params, int layers,
                                                 const float *costT, const float *region,
                                                 const float *adv, float *logp_sorted,
                                                 double *part, double *dE_part)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = P.N, R = P.R;
    const int nacc = acc_count(layers);
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int m = lane & 15, g = lane >> 4;
    const bool two = layers == 2;
    float *W2s = (float *)smem;           // [64][W2S] W2 by output unit
    float *Vs = W2s + 64 * W2S;           // [4][64] W1[:,0], W1[:,1], b2, w3
    float *H1T = Vs + 4 * 64;             // [64][RS] h1 of the chunk's 64 rows, by unit
    float *DLT = H1T + H * RS;            // [64][RS] layer-2 deltas of the chunk, by unit
    float *W1E = DLT + H * RS;            // [64][W1ES] W1's embedding columns
    float *red = W1E + H * W1ES;          // [GW][64] each wave's d1 summed over its rows
    float *prL = red + GW * H;            // [2][64] region term of layer 1, by order parity
    float *ErL = prL + 2 * H;             // [2][16] embedding of the order's region
    float *smx = ErL + 2 * 16;            // [GW] wave softmax max, [GW] sum
    float *crL = smx + 2 * GW;            // [2][N] cost row of the order's region, by parity
    int32_t *x = (int32_t *)(crL + 2 * N); // [N] stock
    float *sbuf = (float *)(x + N);       // [N] scores
    int32_t *sl = (int32_t *)(sbuf + N);  // [N] warehouses with stock
    int32_t *pos = sl + N;                // [N] their index in sl
    int32_t *nfp = pos + N;               // [1] how many
    float *lxs = (float *)(nfp + 4);      // [N] log1p of each warehouse's stock
    const float *W1 = params + (int64_t)R * 16;
    const float b3 = W1[H * 18 + H + (two ? H * H + H : 0) + H];
    stage_w2(W2s, params, R, layers);
    stage_vectors(Vs, params, R, layers);
    for (int i = threadIdx.x; i < H * 16; i += blockDim.x)
        W1E[(i >> 4) * W1ES + (i & 15)] = W1[(i >> 4) * 18 + 2 + (i & 15)];
    // An order's rows that depend on its region only: layer 1's region term, the
    // embedding and the cost row (of the run's trajectory), in slot p & 1 of the LDS
    // copies.  Order p + 1's are loaded into registers when order p starts and written to
    // the other slot before order p's closing barrier (the slot order p - 1 read).
    struct Staged {
        float t, c0, c1; // region term or embedding value (threads < 80); cost row at tid, tid + 256
    };
    auto stage_load = [&](int r, int b) {
        Staged st;
        const int t = threadIdx.x;
        st.t = t < H ? region[(int64_t)r * H + t] : (t < H + 16 ? params[(int64_t)r * 16 + t - H] : 0.f);
        const float *crn = costT + ((int64_t)b * R + r) * N;
        st.c0 = t < N ? crn[t] : 0.f;
        st.c1 = t + 256 < N ? crn[t + 256] : 0.f;
        return st;
    };
    auto stage_store = [&](const Staged &st, int r, int b, int slot) {
        const int t = threadIdx.x;
        if (t < H) prL[slot * H + t] = st.t;
        else if (t < H + 16) ErL[slot * 16 + t - H] = st.t;
        float *cs = crL + slot * N;
        if (t < N) cs[t] = st.c0;
        if (t + 256 < N) cs[t + 256] = st.c1;
        const float *crn = costT + ((int64_t)b * R + r) * N;
        for (int w = t + 512; w < N; w += 256) cs[w] = crn[w];
    };
    // this wave's FP64 record (zeroed before the launch; each value owned by one lane), to
    // which the FP32 sums of every run are added
    double *rec = part + ((int64_t)blockIdx.x * GW + wave) * (nacc + 1);
    const int oW1 = 0, ob1 = H * 18, oW2 = ob1 + H, ob2 = oW2 + (two ? H * H : 0);
    const int ow3 = two ? ob2 + H : ob1 + H, ob3 = ow3 + H;
    const int us = 16 * (m >> 2) + 4 * g + (m & 3); // unit of this lane's scattered sums
    double gobj = 0.0;
    const v4f zero4 = {0.f, 0.f, 0.f, 0.f};
    double *dEw = dE_part + (int64_t)blockIdx.x * R * 16;
    // FP32 sums of this lane's share over the orders since the last flush, added to the
    // wave's FP64 record every FLUSH orders or more (at the end of a run) and at the end
    v4f aW2[4] = {zero4, zero4, zero4, zero4}; // dW2: units o = 16 wave + 4g + v, inputs 16T + m
    float sb1 = 0.f, sw3 = 0.f, sc0 = 0.f, sc1 = 0.f, sb2 = 0.f, sb3 = 0.f;
    float sW1E[4] = {0.f, 0.f, 0.f, 0.f}; // W1[tid / 4][2 + 4 (tid % 4) + k]
    int pending = 0;
    auto flush = [&]() {
        if (two) {
#pragma unroll
            for (int T = 0; T < 4; ++T)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    rec[oW2 + (16 * wave + 4 * g + v) * H + 16 * T + m] += (double)aW2[T][v];
            // db2 of unit 16 wave + m: the four lane groups' row sums, fixed order
            const float p16 = __shfl_xor(sb2, 16, WAVE);
            const float s01 = (lane & 16) ? p16 + sb2 : sb2 + p16;
            const float p32 = __shfl_xor(s01, 32, WAVE);
            const float tb2 = (lane & 32) ? p32 + s01 : s01 + p32;
            if (g == 0) rec[ob2 + 16 * wave + m] += (double)tb2;
        }
        rec[ob1 + us] += (double)sb1;
        rec[oW1 + us * 18] += (double)sc0;
        rec[oW1 + us * 18 + 1] += (double)sc1;
        rec[ow3 + us] += (double)sw3;
        {
            const int i = threadIdx.x >> 2, k0 = 4 * (threadIdx.x & 3);
#pragma unroll
            for (int k = 0; k < 4; ++k) rec[oW1 + i * 18 + 2 + k0 + k] += (double)sW1E[k];
        }
        float t3 = sb3; // lanes of group 0 hold their rows' sums; butterfly in a fixed order
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) t3 += __shfl_xor(t3, d, WAVE);
        if (lane == 0) rec[ob3] += (double)t3;
        aW2[0] = aW2[1] = aW2[2] = aW2[3] = zero4;
        sb1 = sw3 = sc0 = sc1 = sb2 = sb3 = 0.f;
        sW1E[0] = sW1E[1] = sW1E[2] = sW1E[3] = 0.f;
        pending = 0;
    };
    // An order's d1 summed over its rows (each wave's part in red, written before a barrier
    // that every thread has passed since): the embedding columns of dW1 and dE[r].
    bool pend = false; // an order's part in red not yet taken up
    int pend_r = 0, pend_slot = 0;
    double pend_dE = 0.0; // dE[r] of that order as read when it started (wave 0, lanes < 16)
    auto drain = [&]() {
        auto d1o_at = [&](int u) { // fixed order over the waves
            return ((red[u] + red[H + u]) + red[2 * H + u]) + red[3 * H + u];
        };
        {
            const float d = d1o_at(threadIdx.x >> 2);
            const float4 ev = *(const float4 *)(ErL + pend_slot * 16 + 4 * (threadIdx.x & 3));
            sW1E[0] = fmaf(ev.x, d, sW1E[0]);
            sW1E[1] = fmaf(ev.y, d, sW1E[1]);
            sW1E[2] = fmaf(ev.z, d, sW1E[2]);
            sW1E[3] = fmaf(ev.w, d, sW1E[3]);
        }
        if (wave == 0) { // dE[r][k] += sum_j W1[j][2 + k] d1o[j]
            const float d = d1o_at(lane);
            float v[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) v[k] = W1E[lane * W1ES + k] * d;
            float t = reduce_scatter16(v);
            t = t + __shfl_xor(t, 16, WAVE);
            t = t + __shfl_xor(t, 32, WAVE);
            if (lane < 16) dEw[(int64_t)pend_r * 16 + lane] = pend_dE + (double)t;
        }
        pend = false;
    };
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
        // order lo's metadata and rows, and the region of order lo + 1
        int r_cur = 0, a_cur = 0, q_cur = 0, r_nxt = 0;
        float A_cur = 0.f;
        if (lo < hi) {
            r_cur = L.s_region[lo];
            a_cur = L.s_alpha[lo];
            q_cur = L.s_qty[lo];
            A_cur = adv[L.perm[lo]];
        }
        if (lo + 1 < hi) r_nxt = L.s_region[lo + 1];
        __syncthreads(); // (the last run's pending order has been taken up)
        if (lo < hi) stage_store(stage_load(r_cur, b), r_cur, b, lo & 1);
        build_stock_list(x, N, sl, pos, nfp);
        __syncthreads();
        for (int p = lo; p < hi; ++p) {
            if (pend) drain();
            const int r = r_cur, a = a_cur, q = q_cur;
            const float A = A_cur;
            const bool more = p + 1 < hi;
            // order p + 1's metadata (its advantage below, after the scores), the region of
            // order p + 2 and order p + 1's rows, ahead of their use
            int a_n = 0, q_n = 0, pm_n = 0, r_n2 = 0;
            Staged st_n = {0.f, 0.f, 0.f};
            if (more) {
                a_n = L.s_alpha[p + 1];
                q_n = L.s_qty[p + 1];
                pm_n = L.perm[p + 1];
                st_n = stage_load(r_nxt, b);
            }
            if (p + 2 < hi) r_n2 = L.s_region[p + 2];
            float A_n = 0.f;
            const int nf = *nfp;
            const bool bad = a >= 0 ? (a >= N || x[a] <= 0) : nf > 0;
            const float *prO = prL + (p & 1) * H, *ErO = ErL + (p & 1) * 16;
            const float *cr = crL + (p & 1) * N;
            if (!bad && nf > 1) {
                const double dEold = wave == 0 && lane < 16 ? dEw[(int64_t)r * 16 + lane] : 0.0;
                // 1. scores; the first KEEP tiles' activations stay in registers
                const int ntiles = (nf + 15) >> 4;
                v4f k1[KEEP][4], k2[KEEP][4];
                float ks[KEEP], kc[KEEP], kl[KEEP];
                int kw[KEEP];
                float lmx = -INFINITY, lse = 0.f;
#pragma unroll
                for (int j = 0; j < KEEP; ++j) {
                    const int i = (wave + GW * j) * 16 + m;
                    const bool valid = i < nf;
                    const int w = valid ? sl[i] : 0;
                    kw[j] = valid ? w : -1;
                    kc[j] = valid ? cr[w] : 0.f;
                    kl[j] = valid ? lxs[w] : 0.f;
                    if (wave + GW * j < ntiles) {
                        ks[j] = tile_forward(W2s, Vs, two, b3, prO, kc[j], kl[j], k1[j], k2[j]);
                        if (valid) {
                            online_lse(lmx, lse, ks[j]);
                            if (g == 0) sbuf[w] = ks[j];
                        }
                    }
                }
                for (int tile = wave + KEEP * GW; tile < ntiles; tile += GW) {
                    const int i = tile * 16 + m;
                    const bool valid = i < nf;
                    const int w = valid ? sl[i] : 0;
                    v4f h1[4], h2[4];
                    const float sc = tile_forward(W2s, Vs, two, b3, prO, valid ? cr[w] : 0.f,
                                                  valid ? lxs[w] : 0.f, h1, h2);
                    if (valid) {
                        online_lse(lmx, lse, sc);
                        if (g == 0) sbuf[w] = sc;
                    }
                }
                // the wave's partials over the rows of lane group 0 (each row once), fixed order
                {
                    float wmx = g == 0 ? lmx : -INFINITY;
#pragma unroll
                    for (int d = 32; d > 0; d >>= 1) wmx = fmaxf(wmx, __shfl_xor(wmx, d, WAVE));
                    float ws = g == 0 && lmx != -INFINITY ? lse * expf(lmx - wmx) : 0.f;
#pragma unroll
                    for (int d = 32; d > 0; d >>= 1) ws += __shfl_xor(ws, d, WAVE);
                    if (lane == 0) {
                        smx[wave] = wmx;
                        smx[GW + wave] = ws;
                    }
                }
                if (more) A_n = adv[pm_n];
                __syncthreads();
                float mx = -INFINITY;
#pragma unroll
                for (int w = 0; w < GW; ++w) mx = fmaxf(mx, smx[w]);
                float se = 0.f;
#pragma unroll
                for (int w = 0; w < GW; ++w) se += smx[w] == -INFINITY ? 0.f : smx[GW + w] * expf(smx[w] - mx);
                const float lz = logf(se);
                if (threadIdx.x == 0) {
                    const float lp = sbuf[a] - (mx + lz);
                    logp_sorted[p] = lp;
                    gobj += (double)A * (double)lp;
                }
                if (A != 0.f) {
                    float o1 = 0.f; // this order's d1 summed over this wave's rows (scattered)
                    // 2.-3. backward of one tile of this wave (rows past nf: zero deltas)
                    auto backward = [&](const v4f h1[4], const v4f h2[4], float sc, int w,
                                        float cost, float lx, int qc) {
                        const float ds = w >= 0 ? A * ((w == a ? 1.f : 0.f) - expf(sc - mx - lz)) : 0.f;
                        if (g == 0) sb3 += ds;
                        v4f d1[4];
                        float t3[16];
                        if (two) {
                            v4f dl[4];
#pragma unroll
                            for (int t = 0; t < 4; ++t) {
                                const float4 w3v = *(const float4 *)(Vs + 192 + 16 * t + 4 * g);
                                const float w3a[4] = {w3v.x, w3v.y, w3v.z, w3v.w};
#pragma unroll
                                for (int v = 0; v < 4; ++v) {
                                    dl[t][v] = h2[t][v] > 0.f ? ds * w3a[v] : 0.f;
                                    t3[t * 4 + v] = ds * h2[t][v];
                                }
                            }
                            // d1 = [h1 > 0] W2^T dl: A operand W2[o][i] (i = 16T + m, chunk
                            // units o = 16t + 4g + v), B = dl in its D layout
#pragma unroll
                            for (int T = 0; T < 4; ++T) {
                                v4f acc = zero4;
#pragma unroll
                                for (int t = 0; t < 4; ++t) {
                                    const float *wp = W2s + (16 * t + 4 * g) * W2S + 16 * T + m;
                                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wp[0], dl[t][0], acc, 0, 0, 0);
                                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wp[W2S], dl[t][1], acc, 0, 0, 0);
                                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wp[2 * W2S], dl[t][2], acc, 0, 0, 0);
                                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wp[3 * W2S], dl[t][3], acc, 0, 0, 0);
                                }
#pragma unroll
                                for (int v = 0; v < 4; ++v) d1[T][v] = h1[T][v] > 0.f ? acc[v] : 0.f;
                            }
                            // row 16 wave + m of the chunk: in a chunk of qc < 4 tiles at column
                            // 16 (m % 4) + 4 wave + m / 4 (tile t in MFMA steps 4t .. 4t + 3);
                            // in a full chunk at column 16 wave + m (step c: rows c + 16 g),
                            // whose stores fall on distinct banks
                            const int col = qc < GW ? 16 * (m & 3) + 4 * wave + (m >> 2) : 16 * wave + m;
#pragma unroll
                            for (int t = 0; t < 4; ++t)
#pragma unroll
                                for (int v = 0; v < 4; ++v) {
                                    const int at = (16 * t + 4 * g + v) * RS + col;
                                    H1T[at] = h1[t][v];
                                    DLT[at] = dl[t][v];
                                }
                        } else {
#pragma unroll
                            for (int t = 0; t < 4; ++t) {
                                const float4 w3v = *(const float4 *)(Vs + 192 + 16 * t + 4 * g);
                                const float w3a[4] = {w3v.x, w3v.y, w3v.z, w3v.w};
#pragma unroll
                                for (int v = 0; v < 4; ++v) {
                                    d1[t][v] = h1[t][v] > 0.f ? ds * w3a[v] : 0.f;
                                    t3[t * 4 + v] = ds * h1[t][v];
                                }
                            }
                        }
                        // the tile's row sums (scattered over the lanes of each group), one
                        // at a time (kept apart so that their temporaries do not pile up)
                        sw3 += reduce_scatter16(t3);
                        float tt[16];
#pragma unroll
                        for (int t = 0; t < 4; ++t)
#pragma unroll
                            for (int v = 0; v < 4; ++v) tt[t * 4 + v] = d1[t][v];
                        o1 += reduce_scatter16(tt);
                        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                        for (int t = 0; t < 4; ++t)
#pragma unroll
                            for (int v = 0; v < 4; ++v) tt[t * 4 + v] = d1[t][v] * cost;
                        sc0 += reduce_scatter16(tt);
                        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                        for (int t = 0; t < 4; ++t)
#pragma unroll
                            for (int v = 0; v < 4; ++v) tt[t * 4 + v] = d1[t][v] * lx;
                        sc1 += reduce_scatter16(tt);
                    };
                    // dW2 over the rows of the chunk's q tiles (this wave's 16 output units), and
                    // their db2: lane group g reads column block g of the by-unit tensors; with
                    // q < 4 MFMA step c takes rows 4c .. 4c + 3, so tile t is steps 4t .. 4t + 3
                    // and the steps of absent tiles (whose columns hold stale values) are skipped
                    auto chunk_dw2 = [&](int q) {
                        const float4 *ap = (const float4 *)(DLT + (16 * wave + m) * RS + 16 * g);
                        const float4 aq[4] = {ap[0], ap[1], ap[2], ap[3]};
                        float rs = 0.f;
#pragma unroll
                        for (int cb = 0; cb < 4; ++cb)
                            if (cb < q) rs += ((aq[cb].x + aq[cb].y) + aq[cb].z) + aq[cb].w;
                        sb2 += rs;
#pragma unroll
                        for (int T = 0; T < 4; ++T) {
                            const float4 *bp = (const float4 *)(H1T + (16 * T + m) * RS + 16 * g);
#pragma unroll
                            for (int cb = 0; cb < 4; ++cb) {
                                if (cb < q) {
                                    const float4 bq = bp[cb];
                                    aW2[T] = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[cb].x, bq.x, aW2[T], 0, 0, 0);
                                    aW2[T] = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[cb].y, bq.y, aW2[T], 0, 0, 0);
                                    aW2[T] = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[cb].z, bq.z, aW2[T], 0, 0, 0);
                                    aW2[T] = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[cb].w, bq.w, aW2[T], 0, 0, 0);
                                }
                            }
                        }
                    };
                    const int nch = (nf + 63) >> 6;
#pragma unroll
                    for (int j = 0; j < KEEP; ++j) {
                        if (j < nch) {
                            if (wave + GW * j < ntiles)
                                backward(k1[j], k2[j], ks[j], kw[j], kc[j], kl[j], min(GW, ntiles - GW * j));
                            if (two) {
                                __syncthreads();
                                chunk_dw2(min(GW, ntiles - GW * j));
                                if (j + 1 < nch) __syncthreads();
                            }
                        }
                    }
                    for (int j = KEEP; j < nch; ++j) {
                        const int tile = wave + GW * j;
                        if (tile < ntiles) {
                            const int i = tile * 16 + m;
                            const bool valid = i < nf;
                            const int w = valid ? sl[i] : 0;
                            const float cost = valid ? cr[w] : 0.f, lx = valid ? lxs[w] : 0.f;
                            v4f h1[4], h2[4];
                            const float sc = tile_forward(W2s, Vs, two, b3, prO, cost, lx, h1, h2);
                            backward(h1, h2, sc, valid ? w : -1, cost, lx, min(GW, ntiles - GW * j));
                        }
                        if (two) {
                            __syncthreads();
                            chunk_dw2(min(GW, ntiles - GW * j));
                            if (j + 1 < nch) __syncthreads();
                        }
                    }
                    // 4. the order's d1 over all rows, taken up after the order's closing
                    // barrier (at the next order's start or the run's end)
                    sb1 += o1;
                    red[wave * H + us] = o1;
                    pend = true;
                    pend_r = r;
                    pend_slot = p & 1;
                    pend_dE = dEold;
                }
            } else {
                if (more) A_n = adv[pm_n];
                if (threadIdx.x == 0) {
                    if (bad) atomicOr(&L.ctl->error, 8);
                    logp_sorted[p] = 0.f;
                }
                __syncthreads(); // every thread has made the test above
            }
            if (more) stage_store(st_n, r_nxt, b, (p + 1) & 1);
            // the fixed action: every read of this order's state is behind a barrier
            if (threadIdx.x == 0 && a >= 0 && a < N) {
                const int xa = x[a];
                const int nx = xa - (q < xa ? q : xa);
                x[a] = nx;
                lxs[a] = log1p_stock(nx);
                if (xa > 0 && nx == 0) drop_from_list(a, sl, pos, nfp);
            }
            __syncthreads();
            r_cur = r_nxt;
            a_cur = a_n;
            q_cur = q_n;
            A_cur = A_n;
            r_nxt = r_n2;
        }
        if (pend) drain();
        pending += hi - lo;
        if (pending >= FLUSH) flush();
    }
    flush();
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
    return w2_lds_bytes() + vec_lds_bytes() +
           (size_t)(2 * H * RS + H * W1ES + GW * H + 2 * H + 2 * 16 + 2 * GW) * 4 + (size_t)N * 28 + 16;
}

int grad_wg_per_cu(int N) { return 2 * grad_lds(N, 2) <= 160 * 1024 ? 2 : 1; }

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
    const float *region = costT + (int64_t)P.n_traj * P.R * P.N; // setup_costT's region table
    hipLaunchKernelGGL(k_grad, dim3(n_wg), dim3(256), grad_lds(P.N, layers), st, P, L, params,
                       layers, costT, region, adv, logp_sorted, part, dE_part);
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

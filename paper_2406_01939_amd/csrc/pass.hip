// Kernels shared by every pass of the Picard iteration (Algorithm 1), whatever the
// policy: the entry-state scan, the end-of-pass bookkeeping (termination test and the
// restart frontier of Appendix A.3), the consumption of a warm-start cache, and the
// final unpermute.
//
// Entry state.  Under Algorithm 1 a process starts from s_1 and applies the cached
// actions of the steps it does not own (lost sale if the cached warehouse is empty).
// Restricted to one SKU, every such step lowers one warehouse's stock by q, clamped at
// zero, and clamped decrements compose: max(0, max(0, x-a) - b) = max(0, x-a-b).  So a
// run j of a segment starts from max(0, x0 - E_j) with E_j = sum of u_j' over the
// earlier runs j' of the segment, u_j'[w] = sum of q over the run's orders whose cached
// action is w.  E is an exclusive segmented scan of u.
#include "pk_internal.h"

namespace pk {

namespace {

// Split segments are taken 256 at a time per workgroup, strided over the grid (segment
// i goes to workgroup i mod grid, so the long segments of the most frequent SKUs, which
// are neighbours in key order, land in different workgroups): each thread checks one
// segment's frontier, the segments with runs to walk are gathered in LDS, and the
// workgroup then scans them one by one.  A segment's u rows are contiguous; they pass
// through LDS a tile of rows at a time, loaded by the whole workgroup with every load
// in flight, and the exclusive scan down each warehouse's column is done in LDS (one
// thread per column, its running sum carried from tile to tile) and written out as E.
// Runs up to the frontier are final and need no entry state.  The scan resumes at the
// frontier run f from its stored E_f: the previous pass's scan wrote it (f lies past that
// pass's frontier), and no run before f changed since (f is the first run that changed),
// so E_f is still exact.  After the first pass the kernel also lists the runs past the
// frontier (the ones the walk evaluates) in Plan::active.
constexpr int SCAN_TILE = 12288;   // ints of u per LDS tile (48 KB), a multiple of 256
constexpr int SCAN_MAXC = 4;       // columns per thread
static_assert(SCAN_MAXC * 256 >= PK_MAX_WAREHOUSES && SCAN_TILE >= PK_MAX_WAREHOUSES,
              "every warehouse needs a column thread and a tile at least one row");

__global__ __launch_bounds__(256) void k_scan_entry(Prob P, Plan L, int skip_first_pass)
{
    Ctl *ctl = L.ctl;
    if (ctl->done) return;
    const int pass = ctl->pass;
    const int32_t *fprev = L.fr[(pass - 1) & 1];
    int32_t *fcur = L.fr[pass & 1];
    const int n = ctl->n_split_seg;
    const int N = P.N;
    const int32_t *__restrict__ u = L.u;
    int32_t *__restrict__ E = L.E;
    __shared__ int32_t s_g[256], s_f[256];
    __shared__ int32_t s_cnt, s_base;
    __shared__ int32_t tile[SCAN_TILE];
    const int rpt = SCAN_TILE / N; // rows per tile
    unsigned long long n_bytes = 0; // algorithmic HBM bytes (thread 0 counts)
    for (int base = 0; base < n; base += gridDim.x * 256) {
        if (threadIdx.x == 0) s_cnt = 0;
        __syncthreads();
        const int i = base + (int)threadIdx.x * (int)gridDim.x + (int)blockIdx.x;
        if (i < n) {
            const int g = L.split_segs[i];
            const int32_t f = L.no_frontier ? FR_ALL : fprev[g];
            fcur[g] = FR_NONE;
            if (f != FR_NONE && !(pass == 1 && skip_first_pass)) {
                const int k = atomicAdd(&s_cnt, 1);
                s_g[k] = g;
                s_f[k] = f;
            }
        }
        __syncthreads();
        const int cnt = s_cnt;
        if (threadIdx.x == 0) { // every checked segment: its id and frontier read, one write
            const int checked = n - base < gridDim.x * 256 ? (n - base + (int)gridDim.x - 1 -
                                                              (int)blockIdx.x) / (int)gridDim.x
                                                           : 256;
            n_bytes += 12ull * (checked > 0 ? checked : 0);
        }
        for (int t = 0; t < cnt; ++t) {
            const int g = s_g[t];
            const int32_t f = s_f[t];
            const int s0 = L.seg_sr0[g];
            const int nsr = L.seg_sr0[g + 1] - s0;
            if (pass > 1 && !L.no_frontier) { // list the runs this pass walks: j > f
                const int j0 = f + 1;
                const int jc = nsr - j0;
                if (jc > 0) {
                    if (threadIdx.x == 0) s_base = atomicAdd(&ctl->n_active, jc);
                    __syncthreads();
                    for (int k = threadIdx.x; k < jc; k += blockDim.x) L.active[s_base + k] = s0 + j0 + k;
                    __syncthreads();
                }
            }
            const int jmin = f + 1 > 1 ? f + 1 : 1; // runs j > f need E_j; E_0 = 0
            const int64_t row0 = L.sr_uidx[s0];
            // E_f was written by an earlier scan unless this is the first scan after a
            // skipped one (then every run before f is all lost sales and E_f = 0 anyway)
            const bool resume = f >= 1 && !L.no_frontier && (pass > 2 || (pass == 2 && !skip_first_pass));
            const int jstart = resume ? f : 0;
            if (threadIdx.x == 0) // u rows read from jstart, E rows written from jmin, E_f read
                n_bytes += 4ull * N * ((uint64_t)(nsr - jstart) + (nsr > jmin ? nsr - jmin : 0) +
                                       (resume ? 1 : 0)) +
                           (pass > 1 && !L.no_frontier && nsr > f + 1 ? 4ull * (nsr - f - 1) : 0);
            int32_t acc[SCAN_MAXC];
#pragma unroll
            for (int c = 0; c < SCAN_MAXC; ++c) {
                const int w = c * 256 + (int)threadIdx.x;
                acc[c] = resume && w < N ? E[(row0 + f) * N + w] : 0;
            }
            for (int jt = jstart; jt < nsr; jt += rpt) {
                const int nr = nsr - jt < rpt ? nsr - jt : rpt;
                const int nint = nr * N;
                const int32_t *src = u + (row0 + jt) * N;
                { // the tile: all of a thread's loads are issued before its first store
                    int32_t v[SCAN_TILE / 256];
#pragma unroll
                    for (int k = 0; k < SCAN_TILE / 256; ++k) {
                        const int at = k * 256 + (int)threadIdx.x;
                        v[k] = at < nint ? src[at] : 0;
                    }
#pragma unroll
                    for (int k = 0; k < SCAN_TILE / 256; ++k) {
                        const int at = k * 256 + (int)threadIdx.x;
                        if (at < nint) tile[at] = v[k];
                    }
                }
                __syncthreads();
                // exclusive scan down each column, in place
#pragma unroll
                for (int c = 0; c < SCAN_MAXC; ++c) {
                    const int w = c * 256 + (int)threadIdx.x;
                    if (w < N) {
                        int32_t a = acc[c];
                        for (int r0 = 0; r0 < nr; r0 += 8) { // 8 rows' loads, then their sums
                            int32_t v[8];
#pragma unroll
                            for (int k = 0; k < 8; ++k) v[k] = r0 + k < nr ? tile[(r0 + k) * N + w] : 0;
#pragma unroll
                            for (int k = 0; k < 8; ++k) {
                                if (r0 + k < nr) tile[(r0 + k) * N + w] = a;
                                a += v[k];
                            }
                        }
                        acc[c] = a;
                    }
                }
                __syncthreads();
                // E rows j >= jmin of this tile
                const int r0 = jmin > jt ? jmin - jt : 0;
                if (r0 < nr) {
                    int32_t *dst = E + (row0 + jt) * N;
                    for (int at = r0 * N + (int)threadIdx.x; at < nint; at += 256) dst[at] = tile[at];
                }
                __syncthreads();
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && n_bytes)
        atomicAdd(&ctl->stat[blockIdx.x % STAT_SLOTS][ST_SCAN_BYTES], n_bytes);
}

__global__ void k_pass_end(Ctl *ctl)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    pass_end_body(ctl);
}

// u for every run of a split segment from the current cache (warm start).  One wave per
// run; the run's histogram is built in LDS.
__global__ __launch_bounds__(256) void k_consume(Prob P, Plan L)
{
    extern __shared__ int32_t lds[];
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int N = P.N;
    int32_t *h = lds + wave * N;
    const int n = L.ctl->n_split;
    for (int item = blockIdx.x * 4 + wave; item < n; item += gridDim.x * 4) {
        const int s = L.split_list[item];
        for (int w = lane; w < N; w += WAVE) h[w] = 0;
        wave_sync();
        const int lo = L.sr_lo[s], hi = L.sr_lo[s + 1];
        for (int p = lo + lane; p < hi; p += WAVE) {
            const int a = L.s_alpha[p];
            if (a >= 0) atomicAdd(&h[a], L.s_qty[p]);
        }
        wave_sync();
        const int64_t row = L.sr_uidx[s];
        for (int w = lane; w < N; w += WAVE) L.u[row * N + w] = h[w];
        wave_sync();
    }
}

__global__ void k_unpermute(Prob P, Plan L, int32_t *actions, int32_t *shipped)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P.total; p += stride) {
        const int32_t o = L.perm[p];
        actions[o] = L.s_alpha[p];
        if (shipped) shipped[o] = L.s_ship[p];
    }
}

} // namespace

hipError_t launch_scan_entry(const Prob &P, const Plan &L, int n_seg_max, bool skip_first,
                             hipStream_t st)
{
    int grid = (n_seg_max + 255) / 256;
    grid = grid < 1 ? 1 : (grid > 1024 ? 1024 : grid);
    hipLaunchKernelGGL(k_scan_entry, dim3(grid), dim3(256), 0, st, P, L, skip_first ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_pass_end(const Plan &L, hipStream_t st)
{
    hipLaunchKernelGGL(k_pass_end, dim3(1), dim3(64), 0, st, L.ctl);
    return hipGetLastError();
}

hipError_t launch_consume(const Prob &P, const Plan &L, int64_t n_split_max, hipStream_t st)
{
    int64_t g = (n_split_max + 3) / 4;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_consume, dim3((unsigned)g), dim3(256), 4 * P.N * sizeof(int32_t), st, P,
                       L);
    return hipGetLastError();
}

hipError_t launch_unpermute(const Prob &P, const Plan &L, int32_t *actions, int32_t *shipped,
                            hipStream_t st)
{
    int64_t g = (P.total + 255) / 256;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_unpermute, dim3((unsigned)g), dim3(256), 0, st, P, L, actions, shipped);
    return hipGetLastError();
}

} // namespace pk

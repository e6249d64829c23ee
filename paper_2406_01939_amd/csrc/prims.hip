// Device primitives: prefix scan (reduce-then-scan) and a stable LSD radix sort of
// (key, value) pairs, over the whole array or within each segment.  Both serve the
// per-call setup that orders each trajectory's orders by SKU to form the SKU segments and
// process blocks.
#include "pk_internal.h"

namespace pk {

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;
constexpr int SCAN_MID_THREADS = 1024;

template <typename T>
__device__ T block_excl_scan(T v, T *lds_wave, T *total)
{
    // inclusive within the wave
    T x = v;
    for (int d = 1; d < WAVE; d <<= 1) {
        T o = __shfl_up(x, d, WAVE);
        if (__lane_id() >= d) x += o;
    }
    const int wave = threadIdx.x / WAVE, nwaves = blockDim.x / WAVE;
    if (__lane_id() == WAVE - 1) lds_wave[wave] = x;
    __syncthreads();
    T base = 0, tot = 0;
    for (int w = 0; w < nwaves; ++w) {
        T s = lds_wave[w];
        if (w < wave) base += s;
        tot += s;
    }
    __syncthreads();
    if (total) *total = tot;
    return base + x - v;
}

template <typename T>
__global__ __launch_bounds__(SCAN_THREADS) void k_tile_reduce(const T *in, int64_t n, T *partial)
{
    __shared__ T lds[SCAN_THREADS / WAVE];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    T acc = 0;
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t j = base + (int64_t)i * SCAN_THREADS + threadIdx.x;
        if (j < n) acc += in[j];
    }
    for (int d = 32; d > 0; d >>= 1) acc += __shfl_xor(acc, d, WAVE);
    if (__lane_id() == 0) lds[threadIdx.x / WAVE] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T s = 0;
        for (int w = 0; w < SCAN_THREADS / WAVE; ++w) s += lds[w];
        partial[blockIdx.x] = s;
    }
}

// Exclusive scan of the tile partials with one block.
template <typename T>
__global__ __launch_bounds__(SCAN_MID_THREADS) void k_partial_scan(T *partial, int64_t nb)
{
    __shared__ T lds[SCAN_MID_THREADS / WAVE];
    const int64_t per = (nb + SCAN_MID_THREADS - 1) / SCAN_MID_THREADS;
    const int64_t lo = (int64_t)threadIdx.x * per;
    const int64_t hi = lo + per < nb ? lo + per : nb;
    T s = 0;
    for (int64_t i = lo; i < hi; ++i) s += partial[i];
    T total;
    T run = block_excl_scan<T>(s, lds, &total);
    for (int64_t i = lo; i < hi; ++i) {
        T v = partial[i];
        partial[i] = run;
        run += v;
    }
}

template <typename T>
__global__ __launch_bounds__(SCAN_THREADS) void k_tile_scan(T *data, int64_t n, const T *partial,
                                                            int inclusive)
{
    __shared__ T lds[SCAN_THREADS / WAVE];
    __shared__ T stage[SCAN_TILE];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    // coalesced load into LDS, then each thread scans a contiguous run of SCAN_ITEMS
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t j = base + (int64_t)i * SCAN_THREADS + threadIdx.x;
        stage[i * SCAN_THREADS + threadIdx.x] = j < n ? data[j] : T(0);
    }
    __syncthreads();
    T loc[SCAN_ITEMS];
    T s = 0;
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        loc[i] = stage[threadIdx.x * SCAN_ITEMS + i];
        s += loc[i];
    }
    T run = block_excl_scan<T>(s, lds, nullptr) + partial[blockIdx.x];
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        T v = loc[i];
        stage[threadIdx.x * SCAN_ITEMS + i] = inclusive ? run + v : run;
        run += v;
    }
    __syncthreads();
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t j = base + (int64_t)i * SCAN_THREADS + threadIdx.x;
        if (j < n) data[j] = stage[i * SCAN_THREADS + threadIdx.x];
    }
}

template <typename T>
hipError_t scan_impl(T *data, int64_t n, bool inclusive, void *tmp, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    T *partial = (T *)tmp;
    hipLaunchKernelGGL(k_tile_reduce<T>, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, st, data,
                       n, partial);
    hipLaunchKernelGGL(k_partial_scan<T>, dim3(1), dim3(SCAN_MID_THREADS), 0, st, partial, nb);
    hipLaunchKernelGGL(k_tile_scan<T>, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, st, data, n,
                       partial, inclusive ? 1 : 0);
    return hipGetLastError();
}

// ------------------------------------------------------------------ radix sort
// Digits of up to RX_MAXBITS bits (RX_MAXB buckets): a 17-bit key takes two passes.
constexpr int RX_THREADS = 256;
constexpr int RX_CHUNKS = 8;
constexpr int RX_TILE = RX_THREADS * RX_CHUNKS;
constexpr int RX_MAXBITS = 9;
constexpr int RX_MAXB = 1 << RX_MAXBITS;
constexpr int RX_BPT = RX_MAXB / RX_THREADS; // buckets per thread in the per-bucket loops

// A tile's elements and where its per-digit counts live.  Unsegmented: tile t covers
// [t TILE, (t+1) TILE) and digit d's count of tile t sits at d * n_tiles + t.  Segmented
// (segments [seg_off[s], seg_off[s+1]), tile_first[s] their first tile): tiles lie inside
// one segment, and the counts go segment by segment, digit-major within a segment, at
// tile_first[s] * nb + d * (tiles of s) + (t - tile_first[s]); one exclusive scan of that
// layout gives each (tile, digit) its output offset, every segment staying in place.
struct RxTile {
    int64_t lo, hi;       // element range
    int64_t cbase, cstep; // counts index of digit d: cbase + d * cstep
};

template <bool SEG>
__device__ __forceinline__ bool rx_tile(int64_t t, int64_t n, int64_t n_tiles, int nb,
                                        const int64_t *seg_off, const int32_t *tile_first,
                                        int n_seg, RxTile &T)
{
    if (!SEG) {
        T.lo = t * RX_TILE;
        T.hi = T.lo + RX_TILE < n ? T.lo + RX_TILE : n;
        T.cbase = t;
        T.cstep = n_tiles;
        return true;
    }
    __shared__ int s_seg;
    if (t >= tile_first[n_seg]) return false; // past the last tile (launched as a bound)
    if (threadIdx.x == 0) { // the segment holding tile t: last s with tile_first[s] <= t
        int a = 0, b = n_seg - 1;
        while (a < b) {
            const int m = (a + b + 1) / 2;
            if (tile_first[m] <= t) a = m;
            else b = m - 1;
        }
        while (a + 1 < n_seg && tile_first[a + 1] <= t) ++a; // skip empty segments
        s_seg = a;
    }
    __syncthreads();
    const int sg = s_seg;
    const int64_t tf = tile_first[sg];
    const int64_t nt = tile_first[sg + 1] - tf;
    T.lo = seg_off[sg] + (t - tf) * RX_TILE;
    T.hi = T.lo + RX_TILE < seg_off[sg + 1] ? T.lo + RX_TILE : seg_off[sg + 1];
    T.cbase = tf * nb + (t - tf);
    T.cstep = nt;
    return true;
}

template <bool SEG>
__global__ __launch_bounds__(RX_THREADS) void k_radix_count(const int32_t *keys, int64_t n,
                                                            int shift, int bits, int32_t *counts,
                                                            int64_t n_tiles, const int64_t *seg_off,
                                                            const int32_t *tile_first, int n_seg)
{
    __shared__ int32_t hist[RX_MAXB];
    const int nb = 1 << bits, mask = nb - 1;
    RxTile T;
    if (!rx_tile<SEG>(blockIdx.x, n, n_tiles, nb, seg_off, tile_first, n_seg, T)) return;
    for (int k = 0; k < RX_BPT; ++k) hist[k * RX_THREADS + threadIdx.x] = 0;
    __syncthreads();
    for (int c = 0; c < RX_CHUNKS; ++c) {
        int64_t i = T.lo + c * RX_THREADS + threadIdx.x;
        if (i < T.hi) atomicAdd(&hist[(keys[i] >> shift) & mask], 1);
    }
    __syncthreads();
    for (int k = 0; k < RX_BPT; ++k) {
        const int d = k * RX_THREADS + threadIdx.x;
        if (d < nb) counts[T.cbase + (int64_t)d * T.cstep] = hist[d];
    }
}

// Stable scatter: elements of a tile are ranked in index order, 256 at a time; within a
// wave equal digits are matched with one ballot per digit bit, across the 4 waves through
// LDS.
template <bool SEG>
__global__ __launch_bounds__(RX_THREADS) void k_radix_scatter(
    const int32_t *keys, const int32_t *vals, int64_t n, int shift, int bits, const int32_t *offs,
    int64_t n_tiles, int32_t *keys_out, int32_t *vals_out, const int64_t *seg_off,
    const int32_t *tile_first, int n_seg)
{
    __shared__ int32_t s_wcnt[RX_THREADS / WAVE][RX_MAXB];
    __shared__ int32_t s_woff[RX_THREADS / WAVE][RX_MAXB];
    __shared__ int32_t s_run[RX_MAXB];
    __shared__ int32_t s_goff[RX_MAXB];
    const int tid = threadIdx.x, wave = tid / WAVE;
    const int nb = 1 << bits, mask = nb - 1;
    RxTile T;
    if (!rx_tile<SEG>(blockIdx.x, n, n_tiles, nb, seg_off, tile_first, n_seg, T)) return;
    for (int k = 0; k < RX_BPT; ++k) {
        const int d = k * RX_THREADS + tid;
        s_run[d] = 0;
        s_goff[d] = d < nb ? offs[T.cbase + (int64_t)d * T.cstep] : 0;
        for (int w = 0; w < RX_THREADS / WAVE; ++w) s_wcnt[w][d] = 0;
    }
    __syncthreads();
    for (int c = 0; c < RX_CHUNKS; ++c) {
        const int64_t i = T.lo + c * RX_THREADS + tid;
        const bool valid = i < T.hi;
        const int32_t k = valid ? keys[i] : 0;
        const int32_t v = valid ? vals[i] : 0;
        const int d = (k >> shift) & mask;
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < bits; ++b) { // bits is uniform
            const bool bit = (d >> b) & 1;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const int rank = __popcll(peers & lanemask_lt());
        if (valid && rank == 0) s_wcnt[wave][d] = __popcll(peers);
        __syncthreads();
        for (int kk = 0; kk < RX_BPT; ++kk) {
            const int dd = kk * RX_THREADS + tid;
            int run = s_run[dd];
            for (int w = 0; w < RX_THREADS / WAVE; ++w) {
                const int cnt = s_wcnt[w][dd];
                s_woff[w][dd] = run;
                run += cnt;
                s_wcnt[w][dd] = 0;
            }
            s_run[dd] = run;
        }
        __syncthreads();
        if (valid) {
            const int64_t pos = (int64_t)s_goff[d] + s_woff[wave][d] + rank;
            keys_out[pos] = k;
            vals_out[pos] = v;
        }
    }
}

// Tiles per segment (the last entry 0), scanned in place into first tiles.
__global__ void k_seg_tiles(const int64_t *seg_off, int n_seg, int32_t *tile_first)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s > n_seg) return;
    tile_first[s] = s < n_seg ? (int32_t)((seg_off[s + 1] - seg_off[s] + RX_TILE - 1) / RX_TILE) : 0;
}

} // namespace

hipError_t scan_i64(int64_t *data, int64_t n, bool inclusive, void *tmp, hipStream_t st)
{
    return scan_impl<int64_t>(data, n, inclusive, tmp, st);
}

hipError_t scan_i32_excl(int32_t *data, int64_t n, void *tmp, hipStream_t st)
{
    return scan_impl<int32_t>(data, n, false, tmp, st);
}

size_t scan_tmp_bytes(int64_t n)
{
    return (size_t)((n + SCAN_TILE - 1) / SCAN_TILE + 1) * sizeof(int64_t) + 256;
}

size_t radix_tmp_bytes(int64_t n, int n_seg)
{
    const int64_t n_tiles = (n + RX_TILE - 1) / RX_TILE + n_seg;
    const int64_t nc = (int64_t)RX_MAXB * n_tiles;
    return (((size_t)nc * sizeof(int32_t) + 255) & ~(size_t)255) +
           (((size_t)(n_seg + 2) * sizeof(int32_t) + 255) & ~(size_t)255) + scan_tmp_bytes(nc);
}

size_t radix_tmp_bytes(int64_t n) { return radix_tmp_bytes(n, 0); }

int radix_passes(int key_bits)
{
    const int kb = key_bits < 1 ? 1 : key_bits;
    return (kb + RX_MAXBITS - 1) / RX_MAXBITS;
}

// seg_off: nullable device [n_seg + 1] segment bounds (sorted among themselves).
static hipError_t radix_sort_impl(int32_t *keys, int32_t *vals, int32_t *keys_alt,
                                  int32_t *vals_alt, int64_t n, int key_bits, void *tmp,
                                  hipStream_t st, bool *result_in_alt, const int64_t *seg_off,
                                  int n_seg)
{
    *result_in_alt = false;
    if (n <= 1) return hipSuccess;
    const bool seg = seg_off != nullptr && n_seg > 0;
    const int64_t n_tiles = (n + RX_TILE - 1) / RX_TILE + (seg ? n_seg : 0);
    int32_t *counts = (int32_t *)tmp;
    char *rest = (char *)tmp + (((size_t)RX_MAXB * n_tiles * sizeof(int32_t) + 255) & ~(size_t)255);
    int32_t *tile_first = (int32_t *)rest;
    void *scan_tmp = rest + (((size_t)(n_seg + 2) * sizeof(int32_t) + 255) & ~(size_t)255);
    if (seg) {
        hipLaunchKernelGGL(k_seg_tiles, dim3((unsigned)((n_seg + 256) / 256)), dim3(256), 0, st,
                           seg_off, n_seg, tile_first);
        hipError_t e = scan_i32_excl(tile_first, n_seg + 1, scan_tmp, st);
        if (e != hipSuccess) return e;
    }
    int32_t *ki = keys, *vi = vals, *ko = keys_alt, *vo = vals_alt;
    const int passes = radix_passes(key_bits);
    const int kb = key_bits < 1 ? 1 : key_bits;
    const int bits = (kb + passes - 1) / passes; // digit width, <= RX_MAXBITS
    for (int p = 0; p < passes; ++p) {
        const int shift = bits * p;
        // the last digit stops at the key's own bits (the key words may carry other fields
        // above them)
        const int bp = kb - shift < bits ? kb - shift : bits;
        const int64_t nc = ((int64_t)1 << bp) * n_tiles;
        if (seg)
            hipLaunchKernelGGL(k_radix_count<true>, dim3((unsigned)n_tiles), dim3(RX_THREADS), 0,
                               st, ki, n, shift, bp, counts, n_tiles, seg_off, tile_first, n_seg);
        else
            hipLaunchKernelGGL(k_radix_count<false>, dim3((unsigned)n_tiles), dim3(RX_THREADS), 0,
                               st, ki, n, shift, bp, counts, n_tiles, seg_off, tile_first, n_seg);
        hipError_t e = scan_i32_excl(counts, nc, scan_tmp, st);
        if (e != hipSuccess) return e;
        if (seg)
            hipLaunchKernelGGL(k_radix_scatter<true>, dim3((unsigned)n_tiles), dim3(RX_THREADS), 0,
                               st, ki, vi, n, shift, bp, counts, n_tiles, ko, vo, seg_off,
                               tile_first, n_seg);
        else
            hipLaunchKernelGGL(k_radix_scatter<false>, dim3((unsigned)n_tiles), dim3(RX_THREADS), 0,
                               st, ki, vi, n, shift, bp, counts, n_tiles, ko, vo, seg_off,
                               tile_first, n_seg);
        int32_t *t;
        t = ki; ki = ko; ko = t;
        t = vi; vi = vo; vo = t;
        *result_in_alt = !*result_in_alt;
    }
    return hipGetLastError();
}

hipError_t radix_sort_pairs(int32_t *keys, int32_t *vals, int32_t *keys_alt, int32_t *vals_alt,
                            int64_t n, int key_bits, void *tmp, hipStream_t st,
                            bool *result_in_alt)
{
    return radix_sort_impl(keys, vals, keys_alt, vals_alt, n, key_bits, tmp, st, result_in_alt,
                           nullptr, 0);
}

hipError_t radix_sort_pairs_seg(int32_t *keys, int32_t *vals, int32_t *keys_alt,
                                int32_t *vals_alt, int64_t n, int key_bits,
                                const int64_t *seg_off, int n_seg, void *tmp, hipStream_t st,
                                bool *result_in_alt)
{
    return radix_sort_impl(keys, vals, keys_alt, vals_alt, n, key_bits, tmp, st, result_in_alt,
                           seg_off, n_seg);
}

} // namespace pk

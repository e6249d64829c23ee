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
__global__ __launch_bounds__(SCAN_THREADS) void k_tile_scan(const T *src, T *data, int64_t n,
                                                            const T *partial, int inclusive)
{
    __shared__ T lds[SCAN_THREADS / WAVE];
    __shared__ T stage[SCAN_TILE];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    // coalesced load into LDS, then each thread scans a contiguous run of SCAN_ITEMS
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t j = base + (int64_t)i * SCAN_THREADS + threadIdx.x;
        stage[i * SCAN_THREADS + threadIdx.x] = j < n ? src[j] : T(0);
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

// Scan of src into data (src == data: in place).
template <typename T>
hipError_t scan_impl(const T *src, T *data, int64_t n, bool inclusive, void *tmp, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    T *partial = (T *)tmp;
    hipLaunchKernelGGL(k_tile_reduce<T>, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, st, src,
                       n, partial);
    hipLaunchKernelGGL(k_partial_scan<T>, dim3(1), dim3(SCAN_MID_THREADS), 0, st, partial, nb);
    hipLaunchKernelGGL(k_tile_scan<T>, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, st, src, data,
                       n, partial, inclusive ? 1 : 0);
    return hipGetLastError();
}

// ------------------------------------------------------------------ radix sort
// Digits of up to RX_MAXBITS bits (RX_MAXB buckets): a 17-bit key takes two passes.
constexpr int RX_THREADS = 256;
constexpr int RX_CHUNKS = 16;
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
    int seg;              // segmented: the tile's segment
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
        T.seg = 0;
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
    T.seg = sg;
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

// Stable scatter.  Each wave ranks its own contiguous quarter of the tile, 64 elements at
// a time in index order (equal digits matched with one ballot per digit bit), against
// running per-digit counts of its own in LDS, so the waves need no barrier until the tile
// is ranked; then each digit's count per wave becomes a per-wave offset, and every element
// goes to its digit's offset for the tile plus its wave's offset plus its rank.
constexpr int RX_PER_WAVE = RX_TILE / (RX_THREADS / WAVE); // elements per wave and tile
constexpr int RX_ITEMS = RX_PER_WAVE / WAVE;                // per lane

template <bool SEG>
__global__ __launch_bounds__(RX_THREADS) void k_radix_scatter(
    const int32_t *keys, const int32_t *vals, int64_t n, int shift, int bits, const int32_t *offs,
    int64_t n_tiles, int32_t *keys_out, int32_t *vals_out, const int64_t *seg_off,
    const int32_t *tile_first, int n_seg)
{
    __shared__ int32_t s_wcnt[RX_THREADS / WAVE][RX_MAXB]; // per wave: running digit counts
    __shared__ int32_t s_goff[RX_MAXB];
    const int tid = threadIdx.x, wave = tid / WAVE, lane = tid % WAVE;
    const int nb = 1 << bits, mask = nb - 1;
    RxTile T;
    if (!rx_tile<SEG>(blockIdx.x, n, n_tiles, nb, seg_off, tile_first, n_seg, T)) return;
    for (int k = 0; k < RX_BPT; ++k) {
        const int d = k * RX_THREADS + tid;
        s_goff[d] = d < nb ? offs[T.cbase + (int64_t)d * T.cstep] : 0;
        for (int w = 0; w < RX_THREADS / WAVE; ++w) s_wcnt[w][d] = 0;
    }
    __syncthreads();
    const int64_t base = T.lo + (int64_t)wave * RX_PER_WAVE;
    int32_t kr[RX_ITEMS], vr[RX_ITEMS], rk[RX_ITEMS];
#pragma unroll
    for (int c = 0; c < RX_ITEMS; ++c) {
        const int64_t i = base + c * WAVE + lane;
        kr[c] = i < T.hi ? keys[i] : 0;
        vr[c] = i < T.hi ? vals[i] : 0;
    }
    int32_t *cnt = s_wcnt[wave];
#pragma unroll
    for (int c = 0; c < RX_ITEMS; ++c) {
        const int64_t i = base + c * WAVE + lane;
        const bool valid = i < T.hi;
        const int d = (kr[c] >> shift) & mask;
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < bits; ++b) { // bits is uniform
            const bool bit = (d >> b) & 1;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const int rank = __popcll(peers & lanemask_lt());
        const int before = valid ? cnt[d] : 0;
        wave_sync();
        if (valid && rank == 0) cnt[d] = before + __popcll(peers);
        wave_sync();
        rk[c] = before + rank;
    }
    __syncthreads();
    // per digit: the waves' counts into offsets (wave order is index order)
    for (int k = 0; k < RX_BPT; ++k) {
        const int d = k * RX_THREADS + tid;
        int run = 0;
        for (int w = 0; w < RX_THREADS / WAVE; ++w) {
            const int c = s_wcnt[w][d];
            s_wcnt[w][d] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < RX_ITEMS; ++c) {
        const int64_t i = base + c * WAVE + lane;
        if (i < T.hi) {
            const int d = (kr[c] >> shift) & mask;
            const int64_t pos = (int64_t)s_goff[d] + cnt[d] + rk[c];
            keys_out[pos] = kr[c];
            vals_out[pos] = vr[c];
        }
    }
}

// Inverse permutation within segments, in two passes.  perm maps a position p of segment s
// to an index of the same segment; out[perm[p]] = in[p] for two arrays.  First the pairs go
// into key words (index within the segment | (a + 1) << 20) sorted by the index's tile of
// RX_TILE (bits 12 and up, one radix pass within each segment); since perm is a bijection
// within a segment, the pairs bound for its tile t then occupy exactly the positions of
// tile t.  Then each tile is placed through LDS and written out in order.
constexpr int UP_LOW = 12;  // log2(RX_TILE)
constexpr int UP_IDX = 20;  // index bits: segments of at most 2^20 elements
static_assert((1 << UP_LOW) == RX_TILE, "tile of the inverse permutation");

__global__ __launch_bounds__(256) void k_unperm_keys(const int32_t *perm, const int32_t *a,
                                                     const int32_t *b, int64_t n,
                                                     const int64_t *seg_off, int n_seg,
                                                     int32_t *keys, int32_t *vals)
{
    __shared__ int s_seg;
    const int64_t p0 = (int64_t)blockIdx.x * RX_TILE;
    if (p0 >= n) return;
    if (threadIdx.x == 0) s_seg = traj_of(seg_off, n_seg, p0);
    __syncthreads();
    int sg = s_seg;
    const int64_t p1 = p0 + RX_TILE < n ? p0 + RX_TILE : n;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
        while (p >= seg_off[sg + 1]) ++sg;
        const uint32_t idx = (uint32_t)(perm[p] - seg_off[sg]);
        keys[p] = (int32_t)(idx | ((uint32_t)(a[p] + 1) << UP_IDX));
        vals[p] = b ? b[p] : 0;
    }
}

__global__ __launch_bounds__(256) void k_unperm_place(const int32_t *keys, const int32_t *vals,
                                                      int64_t n, const int64_t *seg_off,
                                                      const int32_t *tile_first, int n_seg,
                                                      int64_t n_tiles, int32_t *out_a,
                                                      int32_t *out_b)
{
    __shared__ int32_t sa[RX_TILE], sb[RX_TILE];
    RxTile T;
    if (!rx_tile<true>(blockIdx.x, n, n_tiles, 1, seg_off, tile_first, n_seg, T)) return;
    const int cnt = (int)(T.hi - T.lo);
    for (int j = threadIdx.x; j < cnt; j += blockDim.x) {
        const uint32_t k = (uint32_t)keys[T.lo + j];
        const int at = (int)(k & (RX_TILE - 1));
        sa[at] = (int32_t)(k >> UP_IDX) - 1;
        sb[at] = vals[T.lo + j];
    }
    __syncthreads();
    for (int j = threadIdx.x; j < cnt; j += blockDim.x) {
        out_a[T.lo + j] = sa[j];
        if (out_b) out_b[T.lo + j] = sb[j];
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
    return scan_impl<int64_t>(data, data, n, inclusive, tmp, st);
}

hipError_t scan_i64_to(const int64_t *src, int64_t *dst, int64_t n, bool inclusive, void *tmp,
                       hipStream_t st)
{
    return scan_impl<int64_t>(src, dst, n, inclusive, tmp, st);
}

hipError_t scan_i32_excl(int32_t *data, int64_t n, void *tmp, hipStream_t st)
{
    return scan_impl<int32_t>(data, data, n, false, tmp, st);
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
// Sorts by bits [bit_lo, key_bits) of the keys.
static hipError_t radix_sort_impl(int32_t *keys, int32_t *vals, int32_t *keys_alt,
                                  int32_t *vals_alt, int64_t n, int key_bits, void *tmp,
                                  hipStream_t st, bool *result_in_alt, const int64_t *seg_off,
                                  int n_seg, int bit_lo = 0)
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
    const int kb = key_bits - bit_lo < 1 ? 1 : key_bits - bit_lo; // bits sorted
    const int passes = radix_passes(kb);
    const int bits = (kb + passes - 1) / passes; // digit width, <= RX_MAXBITS
    for (int p = 0; p < passes; ++p) {
        const int shift = bit_lo + bits * p;
        // the last digit stops at the key's own bits (the key words may carry other fields
        // above them)
        const int bp = kb - bits * p < bits ? kb - bits * p : bits;
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

bool unpermute_fits(int64_t longest_segment, int32_t a_max)
{
    return longest_segment <= (1ll << UP_IDX) && a_max + 1 < (1 << (32 - UP_IDX));
}

hipError_t unpermute_seg(const int32_t *perm, const int32_t *a, const int32_t *b, int64_t n,
                         const int64_t *seg_off, int n_seg, int32_t *out_a, int32_t *out_b,
                         int32_t *k0, int32_t *v0, int32_t *k1, int32_t *v1, void *tmp,
                         hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const unsigned g = (unsigned)((n + RX_TILE - 1) / RX_TILE);
    hipLaunchKernelGGL(k_unperm_keys, dim3(g), dim3(256), 0, st, perm, a, b, n, seg_off, n_seg,
                       k0, v0);
    bool alt = false;
    hipError_t e = radix_sort_impl(k0, v0, k1, v1, n, UP_IDX, tmp, st, &alt, seg_off, n_seg,
                                   UP_LOW);
    if (e != hipSuccess) return e;
    const int64_t n_tiles = (n + RX_TILE - 1) / RX_TILE + n_seg;
    const int32_t *tile_first =
        (const int32_t *)((char *)tmp + (((size_t)RX_MAXB * n_tiles * sizeof(int32_t) + 255) &
                                         ~(size_t)255));
    hipLaunchKernelGGL(k_unperm_place, dim3((unsigned)n_tiles), dim3(256), 0, st, alt ? k1 : k0,
                       alt ? v1 : v0, n, seg_off, tile_first, n_seg, n_tiles, out_a, out_b);
    return hipGetLastError();
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

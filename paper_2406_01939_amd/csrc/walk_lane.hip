// The first pass of the greedy Picard walk for short runs: one lane per run.
//
// The first pass walks every run, and most runs are short: a few orders of one SKU inside
// one block.  Walked a wave per run, most of the wave idles and each run pays its set-up
// latency for a few orders.  Here each lane of a wave walks one run, order by order and
// exactly as Algorithm 1's process does (Section 2), and the wave's 64 runs have similar
// lengths (the per-call set-up lists the short runs longest first).  Longer runs stay with
// the wave-per-run walk, launched after this kernel, which also ends the pass.  The length
// limit follows the work: a wave's walk takes as many steps as its longest run, and the
// limit is the number of steps the whole first pass needs when every lane of every wave
// the GPU holds at once walks one order per step (at most LANE_MAX_LEN; below 64 there
// is too little work to fill the GPU and the wave-per-run walk takes every run).
//
// A lane's state is its run's stock row as rem[w] = entry stock minus the units its orders
// have demanded at w so far (unclamped), in LDS as [w][lane]; the stock is max(0, rem).
// The warehouses with stock are a 128-bit set in registers.  The greedy choice (least
// cost, lowest index on ties; Section 3.1) is the first warehouse of the order's region's
// preference list (warehouses in increasing key order of greedy_keys.h) that has stock;
// a lane tests 16 candidates at a time.  An order ships min(q, stock) and lowers rem by q,
// so the final stock is max(0, rem) and the run's cached consumption is entry - rem.
#include <type_traits>

#include "greedy_keys.h"

namespace pk {

namespace {

constexpr int LSTR = WAVE + 1; // LDS words per warehouse row: one per lane and a pad word
constexpr size_t PREF_LDS_MAX = 24576; // preference lists of one trajectory staged in LDS

// Byte offset of the staged preference lists, after the stock rows (16-byte aligned).
__host__ __device__ inline size_t pref_lds_offset(int N)
{
    return ((size_t)N * LSTR * sizeof(int32_t) + 15) & ~(size_t)15;
}

// The stock set: NW 64-bit words (NW = 1 for N <= 64).
template <int NW> struct LaneSet {
    uint64_t w[NW];
    __device__ __forceinline__ bool any() const
    {
        uint64_t o = 0;
#pragma unroll
        for (int i = 0; i < NW; ++i) o |= w[i];
        return o != 0;
    }
    __device__ __forceinline__ uint32_t has(uint32_t v) const
    {
        const uint64_t m = NW == 1 ? w[0] : (v < 64 ? w[0] : w[NW - 1]);
        return (uint32_t)(m >> (v & 63)) & 1u;
    }
    __device__ __forceinline__ void clear(int a)
    {
        if (NW == 1 || a < 64) w[0] &= ~(1ull << (a & 63));
        else w[NW - 1] &= ~(1ull << (a & 63));
    }
};

// Index (0..15) of the first of 16 candidate warehouses (the bytes of v, in order) that
// has stock; 16 if none has.
template <int NW> __device__ __forceinline__ int first_in(uint4 v, const LaneSet<NW> &s)
{
    const uint32_t d[4] = {v.x, v.y, v.z, v.w};
    uint32_t hit = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) hit |= s.has((d[i >> 2] >> (8 * (i & 3))) & 0xffu) << i;
    return hit ? __builtin_ctz(hit) : 16;
}

__device__ __forceinline__ uint32_t comp4(uint4 v, int i)
{
    return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

__device__ __forceinline__ int byte_of(uint4 v, int i)
{
    const uint32_t d = i < 8 ? (i < 4 ? v.x : v.y) : (i < 12 ? v.z : v.w);
    return (int)((d >> (8 * (i & 3))) & 0xffu);
}

__device__ __forceinline__ int wave_max_i(int v)
{
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        const int u = __shfl_xor(v, o, WAVE);
        v = u > v ? u : v;
    }
    return v;
}

// OLD: the call has an initial cache (its old actions are read, and runs after a SKU's
// first enter at x0 - E).  PC: 16-candidate chunks of a preference row loaded ahead per
// order.  NW: stock-set words; with one word (N <= 64) the PC chunks are the whole row,
// with two the later chunks are read when an order needs them.
template <bool OLD, int PC, int NW>
__global__ __launch_bounds__(WAVE) void k_walk_greedy_lane(Prob P, Plan L, int32_t *final_inv)
{
    extern __shared__ int32_t rem[]; // [N][LSTR]
    Ctl *ctl = L.ctl;
    if (ctl->done || ctl->pass != 1) return;
    const int n_lane = ctl->n_lane;
    const int g0 = blockIdx.x * WAVE;
    if (g0 >= n_lane) return;
    const int lane = threadIdx.x;
    const int N = P.N, R = P.R;
    const int npref = pref_npad(N);
    const bool has = g0 + lane < n_lane;
    RunDesc d = {0, 0, 0, 0, 0, 1, -1, 0}; // lanes without a run read position 0, write the sink
    if (has) d = L.rd[L.wlist[ctl->n_wide + g0 + lane]];
    const int lo = d.lo, len = d.hi - d.lo;
    const int b = d.key / P.K;
    const uint8_t *pb = L.pref + (int64_t)b * R * npref;

    // entry rows, 16 runs at a time (the wave reads each row coalesced, every load of the
    // 16 in flight at once); lane k keeps its run's stock set
    LaneSet<NW> fs;
#pragma unroll
    for (int i = 0; i < NW; ++i) fs.w[i] = 0;
    constexpr int EB = 16;
    for (int k0 = 0; k0 < WAVE; k0 += EB) {
        int v[EB][NW];
#pragma unroll
        for (int kk = 0; kk < EB; ++kk) {
            const int k = k0 + kk;
            const int key_k = __builtin_amdgcn_readlane(d.key, k);
            const int32_t *xr = P.x0 + (int64_t)key_k * N;
            bool e_k = false;
            const int32_t *er = xr; // a valid address when the run has no E row
            if (OLD) {
                const int j_k = __builtin_amdgcn_readlane(d.j, k);
                const int u_k = __builtin_amdgcn_readlane(d.uidx, k);
                e_k = j_k > 0;
                if (e_k) er = L.E + (int64_t)u_k * N;
            }
#pragma unroll
            for (int i = 0; i < NW; ++i) {
                const int w = i * WAVE + lane < N ? i * WAVE + lane : N - 1;
                v[kk][i] = xr[w];
                if (OLD) {
                    const int e = er[w];
                    v[kk][i] -= e_k ? e : 0;
                }
            }
        }
#pragma unroll
        for (int kk = 0; kk < EB; ++kk) {
#pragma unroll
            for (int i = 0; i < NW; ++i) {
                const int w = i * WAVE + lane;
                const int x = w < N && v[kk][i] > 0 ? v[kk][i] : 0;
                if (w < N) rem[w * LSTR + k0 + kk] = x;
                const uint64_t m = __ballot(x > 0);
                if (lane == k0 + kk) fs.w[i] = m;
            }
        }
    }
    wave_sync();

    // the walk, in steps aligned to 4-position blocks: step s visits position A0 + s (A0 is
    // lo rounded down to a multiple of 4), so every lane enters a new block at the same
    // step, and a lane's run covers steps [lead, lead + len).  Per block the orders come in
    // one 16-byte load of packed (region, quantity) words (and one of old actions), issued
    // two blocks ahead; the actions and units shipped leave in one 16-byte store per array when
    // the block lies inside the run, else position by position.  The preference row of
    // step s + 4 is loaded at step s.
    const int lead = lo & 3;
    const int A0 = lo - lead;
    const int hi = lo + len;
    const int steps = __builtin_amdgcn_readfirstlane((wave_max_i(has ? lead + len : 0) + 3) & ~3);
    const int rb = L.rq_rb;
    const uint32_t rmask = (1u << rb) - 1u;
    const int64_t nblk = (P.total + 3) >> 2;
    auto blk = [&](int s) -> int64_t {
        const int64_t j = (int64_t)(A0 + s) >> 2;
        return j < nblk ? j : nblk - 1;
    };
    auto region_of = [&](uint32_t w) -> int {
        const int r = (int)(w & rmask);
        return r < R ? r : R - 1; // positions past the run may hold another run's words
    };
    const uint4 *rq4 = (const uint4 *)L.s_rq;
    const uint4 *old4 = (const uint4 *)L.s_alpha;
    // this group's runs all in one trajectory: its preference lists in LDS
    const int b0 = __builtin_amdgcn_readfirstlane(b);
    const bool lds_pref = L.pref_lds && __ballot(has && b != b0) == 0;
    uint8_t *pref_s = (uint8_t *)rem + pref_lds_offset(N);
    if (lds_pref) {
        const uint4 *src = (const uint4 *)(L.pref + (int64_t)b0 * R * npref);
        uint4 *dst = (uint4 *)pref_s;
        const int n16 = R * npref / 16;
        for (int i = lane; i < n16; i += WAVE) dst[i] = src[i];
        wave_sync();
    }
    int nchg = 0;
    auto walk = [&](auto lds_tag) {
        constexpr bool IN_LDS = decltype(lds_tag)::value;
        auto row_of = [&](int r) -> const uint4 * {
            if constexpr (IN_LDS) return (const uint4 *)(pref_s + r * npref);
            else return (const uint4 *)(pb + (int64_t)r * npref);
        };
        // blocks b, b + 1 and b + 2 in Q[b % 3] (the loop below covers three blocks per
        // round, so the roles rotate by name and no register is moved)
        uint4 Q[3], O[3];
        Q[0] = rq4[blk(0)];
        Q[1] = rq4[blk(4)];
        Q[2] = Q[1];
        O[0] = O[1] = O[2] = make_uint4(0, 0, 0, 0);
        if (OLD) {
            O[0] = old4[blk(0)];
            O[1] = old4[blk(4)];
        }
        uint4 pv[4][PC];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint4 *row = row_of(region_of(comp4(Q[0], i)));
#pragma unroll
            for (int c = 0; c < PC; ++c) pv[i][c] = row[c];
        }
        // one stock-set word: the launcher loads the whole row ahead (16 PC >= N)
        constexpr bool whole = NW == 1;
        for (int s00 = 0; s00 < steps; s00 += 12) {
#pragma unroll
            for (int kb = 0; kb < 3; ++kb) {
                const int s0 = s00 + 4 * kb;
                if (s0 < steps) { // wave-uniform
                    const uint4 qc = Q[kb], qn = Q[(kb + 1) % 3];
                    const uint4 oc = O[kb];
                    // the block after next, into the slot this block's words leave
                    Q[(kb + 2) % 3] = rq4[blk(s0 + 8)];
                    if (OLD) O[(kb + 2) % 3] = old4[blk(s0 + 8)];
                    int ab[4], sb[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int s = s0 + i;
                        const bool act = s >= lead && s < lead + len;
                        const uint32_t w = comp4(qc, i);
                        const int r = region_of(w);
                        const int q = (int)(w >> rb);
                        // the first chunk with a warehouse with stock (later chunks only
                        // when some lane of the wave needs them)
                        int a = LOST;
                        bool more = act && fs.any();
#pragma unroll
                        for (int c = 0; c < PC; ++c) {
                            if (c > 0 && !__ballot(more)) break;
                            if (more) {
                                const int h = first_in<NW>(pv[i][c], fs);
                                if (h < 16) {
                                    a = byte_of(pv[i][c], h);
                                    more = false;
                                }
                            }
                        }
                        if (!whole && __ballot(more)) { // the rest of the row, 16 at a time
                            for (int c = PC; c < npref / 16; ++c) {
                                if (!__ballot(more)) break;
                                if (more) {
                                    const uint4 v = row_of(r)[c];
                                    const int h = first_in<NW>(v, fs);
                                    if (h < 16) {
                                        a = byte_of(v, h);
                                        more = false;
                                    }
                                }
                            }
                        }
                        int sh = 0;
                        if (act && a >= 0) {
                            int32_t *rp = &rem[a * LSTR + lane];
                            const int x = *rp;
                            sh = q < x ? q : x;
                            *rp = x - q;
                            if (x <= q) fs.clear(a);
                        }
                        if (act) nchg += a != (OLD ? (int)comp4(oc, i) : LOST);
                        ab[i] = a;
                        sb[i] = sh;
                        // the preference row of step s + 4 (next block, same place)
                        const uint4 *row = row_of(region_of(comp4(qn, i)));
#pragma unroll
                        for (int c = 0; c < PC; ++c) pv[i][c] = row[c];
                    }
                    // the block's results out
                    const int A = A0 + s0;
                    if (has && A >= lo && A + 3 < hi) {
                        *(uint4 *)&L.s_alpha[A] = make_uint4(ab[0], ab[1], ab[2], ab[3]);
                        *(uint4 *)&L.s_ship[A] = make_uint4(sb[0], sb[1], sb[2], sb[3]);
                    } else if (has) {
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            if (A + i >= lo && A + i < hi) {
                                L.s_alpha[A + i] = ab[i];
                                L.s_ship[A + i] = sb[i];
                            }
                        }
                    }
                }
            }
        }
    };
    if (lds_pref) walk(std::true_type{});
    else walk(std::false_type{});
    wave_sync();

    // the run's change marks its segment's frontier (Appendix A.3's restart, per SKU)
    const bool changed = has && nchg > 0;
    if (changed) {
        atomicMin(&L.fr[1][d.g], d.j);
        if (L.traj_lcp[b] < 1) atomicMax(&L.traj_lcp[b], 1);
    }
    if (__ballot(changed) && lane == 0) ctl->any_changed = 1;

    // rows out, one run at a time: the cached consumption (split segments) and the final
    // inventory (a segment's last run)
    int wr = 0; // rows written by this lane's run, for the byte count
    for (int k = 0; k < WAVE; ++k) {
        if (g0 + k >= n_lane) break;
        const int key_k = __builtin_amdgcn_readlane(d.key, k);
        const int j_k = __builtin_amdgcn_readlane(d.j, k);
        const int u_k = __builtin_amdgcn_readlane(d.uidx, k);
        const int nsr_k = __builtin_amdgcn_readlane(d.nsr, k);
        int wk = 0;
        if (u_k >= 0) {
            const int32_t *xr = P.x0 + (int64_t)key_k * N;
            const int32_t *er = (OLD && j_k > 0) ? L.E + (int64_t)u_k * N : nullptr;
            for (int w = lane; w < N; w += WAVE) {
                int e = xr[w] - (er ? er[w] : 0);
                e = e > 0 ? e : 0;
                L.u[(int64_t)u_k * N + w] = e - rem[w * LSTR + k];
            }
            ++wk;
        }
        if (final_inv && j_k == nsr_k - 1) {
            for (int w = lane; w < N; w += WAVE) {
                const int x = rem[w * LSTR + k];
                final_inv[(int64_t)key_k * N + w] = x > 0 ? x : 0;
            }
            ++wk;
        }
        if (lane == k) wr = wk;
    }

    // statistics (the bytes a run moves: per order region and quantity read, action and
    // units shipped written, the old action read with an initial cache; per run its
    // x0 row, its E row when it has one, and the rows it writes)
    const int rows = has ? 1 + ((OLD && d.j > 0) ? 1 : 0) + wr : 0;
    const int by = has ? (OLD ? 20 : 16) * len + 4 * N * rows : 0;
    const int s_orders = wave_sum(has ? len : 0);
    const int s_chg = wave_sum(has ? nchg : 0);
    const int s_bytes = wave_sum(by);
    const int s_runs = __popcll(__ballot(has));
    if (lane == 0) {
        unsigned long long *st = ctl->stat[blockIdx.x % STAT_SLOTS];
        atomicAdd(&st[ST_ORDERS], (unsigned long long)s_orders);
        atomicAdd(&st[ST_RUNS], (unsigned long long)s_runs);
        atomicAdd(&st[ST_CHANGED], (unsigned long long)s_chg);
        atomicAdd(&st[ST_BYTES], (unsigned long long)s_bytes);
    }
}

template <bool OLD, int PC, int NW>
void launch_lane_t(const Prob &P, const Plan &L, int32_t *final_inv, unsigned grid, size_t lds,
                   hipStream_t st)
{
    hipLaunchKernelGGL((k_walk_greedy_lane<OLD, PC, NW>), dim3(grid), dim3(WAVE), lds, st, P, L,
                       final_inv);
}

template <bool OLD>
void launch_lane_n(const Prob &P, const Plan &L, int32_t *final_inv, unsigned grid, size_t lds,
                   hipStream_t st)
{
    // the whole preference row ahead up to N = 64, two chunks beyond
    const int nch = pref_npad(P.N) / 16;
    if (nch <= 1) launch_lane_t<OLD, 1, 1>(P, L, final_inv, grid, lds, st);
    else if (nch == 2) launch_lane_t<OLD, 2, 1>(P, L, final_inv, grid, lds, st);
    else if (nch == 3) launch_lane_t<OLD, 3, 1>(P, L, final_inv, grid, lds, st);
    else if (nch == 4) launch_lane_t<OLD, 4, 1>(P, L, final_inv, grid, lds, st);
    else launch_lane_t<OLD, 2, 2>(P, L, final_inv, grid, lds, st);
}

} // namespace

bool pref_in_lds(int N, int R) { return (size_t)R * pref_npad(N) <= PREF_LDS_MAX; }

size_t walk_lane_lds(int N, int R)
{
    return pref_lds_offset(N) + (pref_in_lds(N, R) ? (size_t)R * pref_npad(N) : 0);
}

int lane_max_for(int64_t total, int N, int R, int n_cus)
{
    // waves a CU holds: its LDS over a wave's share, at most 12 (three per SIMD at the
    // kernel's register count)
    int64_t per_cu = (int64_t)(160 * 1024) / (int64_t)walk_lane_lds(N < 1 ? 1 : N, R);
    per_cu = per_cu < 1 ? 1 : (per_cu > 12 ? 12 : per_cu);
    const int64_t lanes = (int64_t)WAVE * per_cu * (n_cus < 1 ? 1 : n_cus);
    const int64_t m = total / lanes;
    return m < 64 ? 0 : (int)(m > LANE_MAX_LEN ? LANE_MAX_LEN : m); // 0: not worth a launch
}

hipError_t launch_walk_greedy_lane(const Prob &P, const Plan &L, int32_t *final_inv,
                                   bool has_init, int64_t n_list, hipStream_t st)
{
    const int64_t g = (n_list + WAVE - 1) / WAVE;
    const unsigned grid = (unsigned)(g < 1 ? 1 : g);
    const size_t lds = walk_lane_lds(P.N, P.R);
    if (has_init) launch_lane_n<true>(P, L, final_inv, grid, lds, st);
    else launch_lane_n<false>(P, L, final_inv, grid, lds, st);
    return hipGetLastError();
}

} // namespace pk

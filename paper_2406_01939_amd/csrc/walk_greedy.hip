// The Picard run walk under the greedy policy (Section 3.1, inventory as the constraint):
// among warehouses with stock, the least cost[w][region], lowest index on ties; lost
// sale iff none has stock.  The choice is the least key of greedy_keys.h among the
// warehouses with stock.
#include "greedy_keys.h"

namespace pk {

namespace {

constexpr int UNKNOWN = -2;
constexpr int RING_CH = 4;             // chunks of 64 orders in each LDS ring
constexpr int RING = RING_CH * WAVE;   // ring entries

typedef unsigned short pk_u16x2 __attribute__((ext_vector_type(2)));

// A value the whole wave holds alike, handed to the compiler as such (scalar register).
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// The set of warehouses with stock of the run being walked, as a bitmask.  For N <= 128
// its two 64-bit words are wave-uniform values in scalar registers; otherwise the words
// live in LDS with a member count beside them.  With 16-bit keys the set is also kept
// as key masks in LDS: M[d] covers keys 2d (low half) and 2d+1 (high half), all-ones
// for a warehouse without stock, so a masked key is one OR.  clear() takes a
// wave-uniform warehouse.
__device__ __forceinline__ void mask_out(uint32_t *M, int a)
{
    if (M && __lane_id() == 0) M[a >> 1] |= (a & 1) ? 0xffff0000u : 0x0000ffffu;
}
// mask_out for any lane (two warehouses share a mask word: atomic)
__device__ __forceinline__ void mask_out_lane(uint32_t *M, int a)
{
    if (M) atomicOr(&M[a >> 1], (a & 1) ? 0xffff0000u : 0x0000ffffu);
}
// drop() removes, at once, the warehouses of the lanes with emp set (at most one lane per
// warehouse); every lane of the wave calls it.
template <bool SF> struct StockSet;
template <> struct StockSet<true> {
    uint64_t w0 = 0, w1 = 0;
    uint32_t *M = nullptr;
    uint64_t *clr = nullptr; // two zeroed words of LDS
    __device__ __forceinline__ void drop(bool emp, int a)
    {
        if (emp) {
            atomicOr(&clr[a >> 6], 1ull << (a & 63));
            mask_out_lane(M, a);
        }
        wave_sync();
        const uint64_t c0 = clr[0], c1 = clr[1];
        const uint32_t c0l = uni((int)(uint32_t)c0), c0h = uni((int)(uint32_t)(c0 >> 32));
        const uint32_t c1l = uni((int)(uint32_t)c1), c1h = uni((int)(uint32_t)(c1 >> 32));
        w0 &= ~(((uint64_t)c0h << 32) | c0l);
        w1 &= ~(((uint64_t)c1h << 32) | c1l);
        wave_sync();
        if (__lane_id() < 2) clr[__lane_id()] = 0;
    }
    __device__ __forceinline__ uint64_t word(int k) const { return k == 0 ? w0 : w1; }
    __device__ __forceinline__ bool has(int a) const { return ((a < 64 ? w0 : w1) >> (a & 63)) & 1ull; }
    __device__ __forceinline__ bool any() const { return (w0 | w1) != 0; }
    __device__ __forceinline__ void clear(int a)
    {
        if (a < 64) w0 &= ~(1ull << a);
        else w1 &= ~(1ull << (a - 64));
        mask_out(M, a);
    }
};
template <> struct StockSet<false> {
    uint64_t *F = nullptr;
    int32_t *n = nullptr;
    uint32_t *M = nullptr;
    __device__ __forceinline__ uint64_t word(int k) const { return F[k]; }
    __device__ __forceinline__ bool has(int a) const { return (F[a >> 6] >> (a & 63)) & 1ull; }
    __device__ __forceinline__ bool any() const { return *n > 0; }
    __device__ __forceinline__ void clear(int a)
    {
        if (__lane_id() == 0) {
            F[a >> 6] &= ~(1ull << (a & 63));
            *n -= 1;
        }
        mask_out(M, a);
    }
    __device__ __forceinline__ void drop(bool emp, int a)
    {
        const int ne = __popcll(__ballot(emp));
        if (emp) {
            atomicAnd(&F[a >> 6], ~(1ull << (a & 63)));
            mask_out_lane(M, a);
        }
        if (__lane_id() == 0) *n -= ne;
        wave_sync();
    }
};

// Folds 16 keys (32 bytes) into a packed 16-bit minimum, each pair ORed with its mask
// (all-ones halves for warehouses without stock).
__device__ __forceinline__ void fold16(pk_u16x2 &acc, uint4 v0, uint4 v1, uint4 m0, uint4 m1)
{
    const uint32_t d[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
    const uint32_t o[8] = {m0.x, m0.y, m0.z, m0.w, m1.x, m1.y, m1.z, m1.w};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const uint32_t m = d[i] | o[i];
        pk_u16x2 mv;
        __builtin_memcpy(&mv, &m, 4);
        acc = __builtin_elementwise_min(acc, mv);
    }
}

// Least key among the warehouses with stock for one 16-byte aligned row of npad keys;
// the warehouse it names, or LOST if none has stock.  Lanes with need == false only
// follow along.
// N <= 128 (16-bit keys, npad <= 128, stock set in registers): the row is taken in two
// halves of four 16-key chunks; every load of a half is issued before its first fold,
// and chunks whose warehouses have no stock are neither loaded nor folded (wave-uniform
// tests on the stock bits).  Chunks past the row have no stock bits.
__device__ __forceinline__ int least_key_128(const uint16_t *row, const StockSet<true> &fs,
                                             int npad, bool need)
{
    const uint4 *row4 = (const uint4 *)row;
    const uint4 *M4 = (const uint4 *)fs.M;
    pk_u16x2 acc = {0xffff, 0xffff};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint64_t word = fs.word(h); // chunks 4h .. 4h+3
        uint4 v[8], m[8];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int s = 4 * h + c;
            const uint32_t fb = (uint32_t)(word >> (16 * c)) & 0xffffu;
            v[2 * c] = v[2 * c + 1] = m[2 * c] = m[2 * c + 1] = make_uint4(~0u, ~0u, ~0u, ~0u);
            if (fb && s * 16 < npad) { // wave-uniform
                if (need) {
                    v[2 * c] = row4[2 * s];
                    v[2 * c + 1] = row4[2 * s + 1];
                }
                m[2 * c] = M4[2 * s]; // one address for the whole wave
                m[2 * c + 1] = M4[2 * s + 1];
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const uint32_t fb = (uint32_t)(word >> (16 * c)) & 0xffffu;
            if (fb && (4 * h + c) * 16 < npad) fold16(acc, v[2 * c], v[2 * c + 1], m[2 * c], m[2 * c + 1]);
        }
    }
    const uint32_t best = acc.x < acc.y ? acc.x : acc.y;
    return best == 0xffffu ? LOST : (int)(best & 0xffu);
}

// Any N: 32 bytes of keys per step.
template <typename KeyT, typename FS>
__device__ __forceinline__ int least_key(const KeyT *row, const FS &fs, int npad, bool need)
{
    const uint4 *row4 = (const uint4 *)row;
    constexpr int PER = 16 / (int)sizeof(KeyT); // keys per 16 bytes
    constexpr int STEP = 2 * PER;               // keys per step (divides 64)
    if constexpr (sizeof(KeyT) == 2) {
        pk_u16x2 acc = {0xffff, 0xffff};
        for (int base = 0; base < npad; base += STEP) {
            const uint32_t fb = (uint32_t)(fs.word(base >> 6) >> (base & 63)) & 0xffffu;
            if (fb == 0) continue; // wave-uniform
            const uint4 *M4 = (const uint4 *)fs.M;
            if (need) fold16(acc, row4[base / PER], row4[base / PER + 1], M4[base / PER], M4[base / PER + 1]);
        }
        const uint32_t best = acc.x < acc.y ? acc.x : acc.y;
        return best == 0xffffu ? LOST : (int)(best & 0xffu);
    } else {
        uint32_t acc = 0xffffffffu;
        for (int base = 0; base < npad; base += STEP) {
            const uint32_t fb = (uint32_t)(fs.word(base >> 6) >> (base & 63)) & 0xffu;
            if (fb == 0) continue;
            if (need) {
                const uint4 v0 = row4[base / PER], v1 = row4[base / PER + 1];
                const uint32_t d[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const uint32_t m = ((fb >> i) & 1u) ? d[i] : 0xffffffffu;
                    acc = m < acc ? m : acc;
                }
            }
        }
        return acc == 0xffffffffu ? LOST : (int)(acc & 0xffffu);
    }
}

template <typename KeyT, bool SF>
__device__ __forceinline__ int choose(const KeyT *row, const StockSet<SF> &fs, int npad, bool need)
{
    if constexpr (SF && sizeof(KeyT) == 2) return least_key_128((const uint16_t *)row, fs, npad, need);
    else return least_key<KeyT>(row, fs, npad, need);
}

// One wave walks one run (a process's orders of one SKU) from its entry state, exactly
// as Algorithm 1's process does, 64 orders at a time:
//  * every lane takes the choice its order would get at the step's starting state;
//  * a warehouse whose stock does not exceed the step's demand may empty inside the
//    step: the step's demand per warehouse is summed in LDS, and for a warehouse whose
//    demand exceeds its stock the first order that finds it empty (earlier demand on it
//    >= its stock) is the first order whose choice is no longer valid;
//  * all orders before the first such order are exact (stock only falls, so a choice
//    changes only when the chosen warehouse empties); they are committed and the walk
//    resumes there.
// When every chosen warehouse has more stock than the step's whole demand nothing can
// empty and the step commits without further checks.
// Choices: each region's choice is memoised and recomputed (least key over the stock
// set) only when its warehouse has emptied.  For long runs every region's memo is
// filled up front.
// Orders in: the run is read in 64-order chunks into registers, two chunks at a time and
// two chunks ahead of use (a load has about two steps to arrive), and both are put into
// a 256-entry ring in LDS when the walk reaches the first of them; a step reads its 64
// orders from the ring at any offset.  Actions out: committed actions and shipped units
// go to a second 256-entry ring and leave for global memory two whole chunks at a time.  The next run's descriptor is loaded while the current run is walked.
// The key table of the run's trajectory is read from LDS (one copy per workgroup for a
// single trajectory, one per wave for small tables) or from global memory.
// Per wave LDS: lm[N] (64-bit: the step's lanes per warehouse for unit demand; as int32,
// the step's demand per warehouse otherwise; zero between steps), x[N] stock, cons[N] run
// consumption (unclamped, for u), bw[R] memo, member count, F[ceil(N/64)] and two
// zeroed words, key masks M (16-bit keys), in-ring[256] (region | (old+1) << 12, qty),
// out-ring[256] (action, shipped).
template <typename KeyT> __host__ __device__ inline size_t mask_bytes(int N)
{
    return sizeof(KeyT) == 2 ? (size_t)tab_npad<KeyT>(N) * 2 : 0; // one bit pattern per key
}
template <typename KeyT> __host__ __device__ inline size_t walk_wave_bytes(int N, int R, int mode)
{
    const size_t tb = (size_t)tab_stride<KeyT>(N, R) * sizeof(KeyT);
    const size_t ints = ((size_t)8 * N + (size_t)(2 * N + R + 1) * 4 + 15) & ~(size_t)15;
    const size_t f = ((size_t)8 * ((N + 63) / 64) + 16 + 15) & ~(size_t)15;
    return (mode == 1 ? tb : 0) + ints + f + mask_bytes<KeyT>(N) + 2 * RING * sizeof(int2);
}

__device__ __forceinline__ int2 pack_in(int r, int q, int old) { return make_int2(r | ((old + 1) << 12), q); }

template <typename KeyT, int TABMODE, bool SF, int WPB> // TABMODE 0: global table, 1: per-wave
                                                        // LDS, 2: per-WG LDS; SF: stock set in
                                                        // registers; WPB waves per workgroup
__global__ __launch_bounds__(WPB * 64) void k_walk_greedy(Prob P, Plan L, const KeyT *key_g,
                                                     int32_t *final_inv, int has_init,
                                                     int32_t *sink)
{
    extern __shared__ __align__(16) unsigned char smem[];
    // wave-uniform values are made visible to the compiler as such, so the walk's control
    // flow is scalar branches and its waits count only what is outstanding
    const int wave = uni(threadIdx.x / WAVE), lane = threadIdx.x % WAVE;
    const int N = P.N, R = P.R;
    const int nw = (N + 63) / 64;
    const int npad = tab_npad<KeyT>(N);
    const size_t tab_bytes = (size_t)tab_stride<KeyT>(N, R) * sizeof(KeyT);
    const size_t ints_bytes = ((size_t)8 * N + (size_t)(2 * N + R + 1) * 4 + 15) & ~(size_t)15;
    const size_t f_bytes = ((size_t)8 * nw + 16 + 15) & ~(size_t)15;
    unsigned char *wb = smem + (TABMODE == 2 ? tab_bytes : 0) +
                        wave * walk_wave_bytes<KeyT>(N, R, TABMODE);
    KeyT *wtab = (KeyT *)wb;
    const size_t ints_off = TABMODE == 1 ? tab_bytes : 0;
    uint64_t *lm = (uint64_t *)(wb + ints_off);
    int32_t *tot = (int32_t *)lm;
    int32_t *x = (int32_t *)(lm + N);
    int32_t *cons = x + N;
    int32_t *bw = cons + N;
    int32_t *nfeas = bw + R;
    uint64_t *F = (uint64_t *)(wb + ints_off + ints_bytes);
    uint64_t *clr = F + nw;
    if (lane < 2) clr[lane] = 0;
    uint32_t *M = sizeof(KeyT) == 2 ? (uint32_t *)(wb + ints_off + ints_bytes + f_bytes) : nullptr;
    int2 *ring = (int2 *)(wb + ints_off + ints_bytes + f_bytes + mask_bytes<KeyT>(N));
    int2 *oring = ring + RING;
    Ctl *ctl = L.ctl;
    if (ctl->done) return;
    if (TABMODE == 2) { // one trajectory: its table, once per workgroup
        const uint4 *src = (const uint4 *)key_g;
        uint4 *dst = (uint4 *)smem;
        const int n16 = (int)(tab_bytes / 16);
        for (int i = threadIdx.x; i < n16; i += blockDim.x) dst[i] = src[i];
        __syncthreads();
    }
    int tab_b = -1;
    const int pass = ctl->pass;
    int32_t *fcur = L.fr[pass & 1];
    // pass 1 (and the no-frontier mode) walks every run; later passes walk the runs past
    // each SKU's frontier, listed by the entry scan.  With a first-pass list, pass 1 walks
    // only its long runs here (the lane walk has taken the others).
    const bool all = pass == 1 || L.no_frontier;
    const bool head = pass == 1 && L.wlist != nullptr;
    const int n_items = head ? ctl->n_wide : (all ? ctl->n_sr : ctl->n_active);
    const bool need_E = pass > 1 || has_init;
    int lcp_b = -1; // last trajectory this wave marked as changed in this pass
    unsigned long long n_orders = 0, n_runs = 0, n_changed = 0, n_bytes = 0;

    // static round-robin over the runs (no shared work counter: one hot address), across
    // workgroups first, so that a few long runs of a late pass land on different CUs
    const int n_waves = gridDim.x * WPB;
    int item = wave * gridDim.x + blockIdx.x;
    RunDesc d = {};
    if (item < n_items) d = L.rd[head ? L.wlist[item] : (all ? item : L.active[item])];
    for (; item < n_items; item += n_waves) {
        const int lo = uni(d.lo), hi = uni(d.hi), key = uni(d.key), g = uni(d.g);
        const int j = uni(d.j), nsr = uni(d.nsr), uidx = uni(d.uidx);
        const int b = key / P.K;
        const int nxt = item + n_waves;
        const int s_next = nxt < n_items ? (head ? L.wlist[nxt] : (all ? nxt : L.active[nxt])) : -1;
        // the run's first chunk (loads clamped into the run)
        const int nch = (hi - lo + WAVE - 1) / WAVE;
        const int i0 = lo + lane < hi ? lo + lane : hi - 1;
        const int r0 = L.s_region[i0], q0 = L.s_qty[i0], o0 = L.s_alpha[i0];
        const int32_t *x0row = P.x0 + (int64_t)key * N;
        const int32_t *Erow = (need_E && j > 0) ? L.E + (int64_t)uidx * N : nullptr;
        const KeyT *tab;
        if (TABMODE == 0) {
            tab = key_g + b * tab_stride<KeyT>(N, R);
        } else if (TABMODE == 1) {
            if (b != tab_b) { // this wave's copy of the run's trajectory table
                const uint4 *src = (const uint4 *)(key_g + b * tab_stride<KeyT>(N, R));
                uint4 *dst = (uint4 *)wtab;
                const int n16 = (int)(tab_bytes / 16);
                for (int i = lane; i < n16; i += WAVE) dst[i] = src[i];
                tab_b = b;
            }
            tab = wtab;
        } else {
            tab = (const KeyT *)smem;
        }
        StockSet<SF> fs;
        int nf = 0;
        for (int k = 0; k < nw; ++k) {
            const int w = k * WAVE + lane;
            int32_t v = 0;
            if (w < N) {
                v = x0row[w] - (Erow ? Erow[w] : 0);
                v = v > 0 ? v : 0;
                x[w] = v;
                lm[w] = 0;
                cons[w] = 0;
            }
            const uint64_t m = __ballot(v > 0);
            if constexpr (SF) {
                if (k == 0) fs.w0 = m;
                else fs.w1 = m;
            } else {
                if (lane == 0) F[k] = m;
            }
            nf += __popcll(m);
        }
        if constexpr (!SF) {
            fs.F = F;
            fs.n = nfeas;
            if (lane == 0) *nfeas = nf;
            wave_sync();
        }
        fs.M = M;
        if constexpr (SF) fs.clr = clr;
        if (M) { // key masks from the stock set
            for (int dd = lane; dd < npad / 2; dd += WAVE) {
                const int w = 2 * dd;
                const bool s0 = w < N && fs.has(w), s1 = w + 1 < N && fs.has(w + 1);
                M[dd] = (s0 ? 0u : 0x0000ffffu) | (s1 ? 0u : 0xffff0000u);
            }
        }
        ring[lane] = pack_in(r0, q0, o0); // chunk 0
        RunDesc dn = {}; // the next run's descriptor
        if (s_next >= 0) dn = L.rd[s_next];
        // chunks 1 and 2 into the prefetch registers, followed by four stores to the
        // sink: the same operations, in the same order, as every advance below, so the
        // wait for the prefetch registers counts the same outstanding operations on every
        // path
        __builtin_amdgcn_sched_barrier(0);
        const int i1 = lo + WAVE + lane < hi ? lo + WAVE + lane : hi - 1;
        const int i2 = lo + 2 * WAVE + lane < hi ? lo + 2 * WAVE + lane : hi - 1;
        int rs = L.s_region[i1], qs = L.s_qty[i1], os = L.s_alpha[i1];
        int rs2 = L.s_region[i2], qs2 = L.s_qty[i2], os2 = L.s_alpha[i2];
        sink[2 * WAVE + lane] = 0; // four stores to four places (none merged away)
        sink[3 * WAVE + lane] = 0;
        sink[lane] = 0;
        sink[WAVE + lane] = 0;
        __builtin_amdgcn_sched_barrier(0);
        int cw = 1; // chunks in the in-ring
        int fl = 0; // chunks of actions already out
        wave_sync();
        if (hi - lo >= 2 * WAVE) { // long run: every region's choice up front
            for (int rb0 = 0; rb0 < R; rb0 += WAVE) {
                const int rr = rb0 + lane;
                const bool mine = rr < R;
                const int c = choose<KeyT, SF>(tab + (int64_t)(mine ? rr : 0) * npad, fs, npad, mine);
                if (mine) bw[rr] = c;
            }
        } else {
            for (int rr = lane; rr < R; rr += WAVE) bw[rr] = UNKNOWN;
        }
        wave_sync();
        bool changed = false;
        int p = lo;
        while (p < hi) {
            p = uni(p);
            cw = uni(cw);
            const int off = p - lo;
            // the step reads positions off .. off+63: chunks up to (off + 63) / 64
            const int need_c = (off + WAVE - 1) / WAVE + 1 < nch ? (off + WAVE - 1) / WAVE + 1 : nch;
            if (cw < need_c) { // at most one new chunk per step (a step advances <= 64)
                // chunks cw and cw+1 (loaded at the previous advance) into the ring, then
                // chunks cw+2 and cw+3 into the same registers (written before they are
                // reloaded: no copies of registers whose loads are in flight).  The ring
                // then holds chunks cw-1 .. cw+1 (the step reads from chunk cw-1 on).
                ring[(cw & (RING_CH - 1)) * WAVE + lane] = pack_in(rs, qs, os);
                ring[((cw + 1) & (RING_CH - 1)) * WAVE + lane] = pack_in(rs2, qs2, os2);
                __builtin_amdgcn_sched_barrier(0);
                const int pc = lo + (cw + 2) * WAVE + lane;
                const int ic = pc < hi ? pc : hi - 1;
                const int ic2 = pc + WAVE < hi ? pc + WAVE : hi - 1;
                rs = L.s_region[ic];
                qs = L.s_qty[ic];
                os = L.s_alpha[ic];
                rs2 = L.s_region[ic2];
                qs2 = L.s_qty[ic2];
                os2 = L.s_alpha[ic2];
                // chunks cw-3 and cw-2 are committed in full: out to global memory
                // (stored to the sink before there are any, so every advance issues the
                // same operations; both precede chunk cw-1 < the last chunk: full)
#pragma unroll
                for (int k = 3; k >= 2; --k) {
                    const int c = cw - k;
                    const int po = lo + c * WAVE + lane;
                    const int2 o = oring[(c * WAVE + lane) & (RING - 1)];
                    int32_t *pa = c >= 0 ? &L.s_alpha[po] : &sink[(2 * (k - 2)) * WAVE + lane];
                    int32_t *ps = c >= 0 ? &L.s_ship[po] : &sink[(2 * (k - 2) + 1) * WAVE + lane];
                    *pa = o.x;
                    *ps = o.y;
                }
                fl = cw - 1;
                cw += 2;
                wave_sync();
            }
            const int n = hi - p < WAVE ? hi - p : WAVE;
            const bool act = lane < n;
            const int2 e = ring[(off + lane) & (RING - 1)];
            const int r = act ? (e.x & 0xfff) : 0, q = act ? e.y : 0, old = (e.x >> 12) - 1;
            int a = LOST;
            if (fs.any()) {
                bool need = false;
                if (act) {
                    a = bw[r];
                    need = a == UNKNOWN || (a >= 0 && !fs.has(a));
                }
                if (__ballot(need)) {
                    const int c = choose<KeyT, SF>(tab + (int64_t)r * npad, fs, npad, need);
                    if (need) {
                        a = c;
                        bw[r] = c;
                    }
                }
            }
            wave_sync();
            const bool chose = act && a >= 0;
            const int xa = chose ? x[a] : 0;
            // a chosen warehouse can empty in this step only if its stock does not exceed
            // the step's demand
            const bool unit = __ballot(act && q != 1) == 0;
            const int demand = unit ? n : wave_sum(q);
            const bool risky = __ballot(chose && xa <= demand) != 0;
            int cut = n;
            int ship = q;
            int ta = 0;
            bool over = false; // some warehouse's demand in this step exceeds its stock
            uint64_t mk = 0;   // unit demand: the step's lanes on this lane's warehouse
            int rank = 0;      // unit demand: earlier lanes on this lane's warehouse
            if (risky && unit) {
                // the lanes on each chosen warehouse as one 64-bit mask, built with
                // order-free atomic ORs; an order finds its warehouse empty iff the
                // number of earlier lanes on it reaches the stock
                if (chose) atomicOr(&lm[a], 1ull << lane);
                wave_sync();
                mk = chose ? lm[a] : 0ull;
                wave_sync();
                if (chose) lm[a] = 0ull;
                rank = __popcll(mk & lanemask_lt());
                const uint64_t inv = __ballot(chose && rank >= xa);
                over = inv != 0;
                if (over) cut = __ffsll((long long)inv) - 1;
            } else if (risky) {
                if (chose) atomicAdd(&tot[a], q);
                wave_sync();
                ta = chose ? tot[a] : 0;
                uint64_t todo = __ballot(chose && ta > xa);
                over = todo != 0;
                while (todo) {
                    const int l0 = __ffsll((long long)todo) - 1;
                    const int w0 = __builtin_amdgcn_readlane(a, l0);
                    const bool mine = chose && a == w0;
                    const uint64_t eq = __ballot(mine);
                    int excl;
                    if (unit) {
                        excl = __popcll(eq & lanemask_lt()); // demand of earlier lanes on w0
                    } else {
                        const int qq = mine ? q : 0;
                        excl = wave_incl_sum(qq) - qq;
                    }
                    const int xw = __builtin_amdgcn_readlane(xa, l0);
                    const bool invalid = mine && excl >= xw;
                    if (mine && !invalid) ship = q < xw - excl ? q : xw - excl;
                    const uint64_t inv = __ballot(invalid);
                    if (inv) {
                        const int c = __ffsll((long long)inv) - 1;
                        cut = c < cut ? c : cut;
                    }
                    todo &= ~eq;
                }
            }
            if (risky) {
                cut = uni(cut);
                if (cut == 0) {
                    // the first order's warehouse is in the stock set yet has no stock:
                    // the walk's state is inconsistent; report it instead of spinning
                    if (lane == 0) {
                        atomicOr(&ctl->error, ERR_NO_PROGRESS);
                        ctl->done = 2;
                    }
                    break;
                }
            }
            const bool commit = act && lane < cut;
            const bool chg = commit && a != old;
            changed |= chg;
            n_changed += __popcll(__ballot(chg));
            const int sh = a >= 0 ? ship : 0;
            if (commit) oring[(off + lane) & (RING - 1)] = make_int2(a, sh);
            if (risky && unit) {
                // each warehouse's first lane applies the step's committed demand on it
                // (orders past the stock are past the cut, so it never exceeds the stock)
                const uint64_t cm = cut >= WAVE ? ~0ull : ((1ull << cut) - 1ull);
                const int cnt = __popcll(mk & cm);
                if (chose && rank == 0) {
                    x[a] = xa - cnt;
                    atomicAdd(&cons[a], cnt);
                }
                // the committed order that takes a warehouse's last unit empties it
                const bool emp = commit && chose && rank == xa - 1;
                if (__ballot(emp)) fs.drop(emp, a);
            } else if (risky) {
                uint64_t em;
                if (!over) {
                    // no warehouse's demand exceeds its stock: every order ships in full
                    // and a warehouse empties iff the demand on it equals its stock
                    if (chose) {
                        atomicSub(&x[a], sh);
                        atomicAdd(&cons[a], q);
                    }
                    em = __ballot(chose && ta == xa);
                } else {
                    bool emptied = false;
                    if (commit && a >= 0) {
                        const int before = atomicSub(&x[a], sh);
                        emptied = before == sh; // this order took the last unit
                        atomicAdd(&cons[a], q);
                    }
                    em = __ballot(emptied);
                }
                if (chose) tot[a] = 0;
                while (em) { // wave-uniform: each emptied warehouse leaves the stock set
                    const int l0 = __ffsll((long long)em) - 1;
                    const int w0 = __builtin_amdgcn_readlane(a, l0);
                    fs.clear(w0);
                    em &= ~__ballot(chose && a == w0);
                }
            } else if (commit && a >= 0) {
                atomicSub(&x[a], sh);
                atomicAdd(&cons[a], q);
            }
            wave_sync();
            p += cut;
        }
        // the last (at most three) chunks of actions
        for (int c = fl; c < nch; ++c) {
            const int po = lo + c * WAVE + lane;
            const int2 o = oring[(c * WAVE + lane) & (RING - 1)];
            int32_t *pa = po < hi ? &L.s_alpha[po] : &sink[lane];
            int32_t *ps = po < hi ? &L.s_ship[po] : &sink[WAVE + lane];
            *pa = o.x;
            *ps = o.y;
        }
        wave_sync();
        int wr = 0;
        if (uidx >= 0) {
            for (int w = lane; w < N; w += WAVE) L.u[(int64_t)uidx * N + w] = cons[w];
            ++wr;
        }
        if (final_inv && j == nsr - 1) {
            for (int w = lane; w < N; w += WAVE) final_inv[(int64_t)key * N + w] = x[w];
            ++wr;
        }
        const bool any = __ballot(changed) != 0;
        if (lane == 0) {
            if (any) {
                atomicMin(&fcur[g], j);
                if (b != lcp_b) { // once per trajectory and wave; read first (one hot word)
                    if (L.traj_lcp[b] < pass) atomicMax(&L.traj_lcp[b], pass);
                    lcp_b = b;
                }
            }
            n_orders += hi - lo;
            n_runs += 1;
            n_bytes += 20ull * (hi - lo) + 4ull * N * (1 + (Erow ? 1 : 0) + wr);
        }
        wave_sync();
        d = dn;
    }
    if (lane == 0 && n_runs) {
        unsigned long long *st = ctl->stat[(blockIdx.x * WPB + wave) % STAT_SLOTS];
        atomicAdd(&st[ST_ORDERS], n_orders);
        atomicAdd(&st[ST_RUNS], n_runs);
        atomicAdd(&st[ST_CHANGED], n_changed);
        atomicAdd(&st[ST_BYTES], n_bytes);
    }
    walk_finish(ctl, lcp_b >= 0);
}

struct WalkCfg {
    int mode;
    size_t lds;
    int wpb; // waves per workgroup
};

// LDS per CU (gfx950).
constexpr size_t CU_LDS = 160 * 1024;

// One trajectory: its table once per workgroup, with 16 waves sharing it when they fit in
// a CU's LDS (one workgroup per CU), else 4.  Batches: one table copy per wave when tables
// are small, else the table in global memory; 4 waves per workgroup.
template <typename KeyT> WalkCfg walk_cfg_t(int N, int R, int n_traj)
{
    const size_t tb = (size_t)tab_stride<KeyT>(N, R) * sizeof(KeyT);
    const size_t per = walk_wave_bytes<KeyT>(N, R, 0);
    const size_t per1 = walk_wave_bytes<KeyT>(N, R, 1);
    if (n_traj == 1 && tb + 16 * per <= CU_LDS) return {2, tb + 16 * per, 16};
    if (n_traj == 1 && tb + 4 * per <= 64 * 1024) return {2, tb + 4 * per, 4};
    if (tb <= 8 * 1024 && 4 * per1 <= 64 * 1024) return {1, 4 * per1, 4};
    return {0, 4 * per, 4};
}

template <typename KeyT, bool SF>
void launch_walk_t(const Prob &P, const Plan &L, const void *keys, int32_t *final_inv, int hi,
                   int n_cus, hipStream_t st)
{
    const WalkCfg c = walk_cfg_t<KeyT>(P.N, P.R, P.n_traj);
    const KeyT *t = (const KeyT *)keys;
    if (c.mode == 2 && c.wpb == 16) // one workgroup per CU
        hipLaunchKernelGGL((k_walk_greedy<KeyT, 2, SF, 16>), dim3(n_cus), dim3(1024), c.lds, st,
                           P, L, t, final_inv, hi, L.sink);
    else if (c.mode == 2)
        hipLaunchKernelGGL((k_walk_greedy<KeyT, 2, SF, 4>), dim3(n_cus * 8), dim3(256), c.lds, st,
                           P, L, t, final_inv, hi, L.sink);
    else if (c.mode == 1)
        hipLaunchKernelGGL((k_walk_greedy<KeyT, 1, SF, 4>), dim3(n_cus * 8), dim3(256), c.lds, st,
                           P, L, t, final_inv, hi, L.sink);
    else
        hipLaunchKernelGGL((k_walk_greedy<KeyT, 0, SF, 4>), dim3(n_cus * 8), dim3(256), c.lds, st,
                           P, L, t, final_inv, hi, L.sink);
}

inline bool keys16_n(int N) { return N <= 255; } // as keys16: 0xffff means no stock

} // namespace

size_t walk_greedy_lds(int N, int R)
{
    return keys16_n(N) ? walk_cfg_t<uint16_t>(N, R, 2).lds : walk_cfg_t<uint32_t>(N, R, 2).lds;
}

hipError_t launch_walk_greedy(const Prob &P, const Plan &L, const void *keys, int32_t *final_inv,
                              bool has_init, int n_cus, hipStream_t st)
{
    if (P.N <= 128)
        launch_walk_t<uint16_t, true>(P, L, keys, final_inv, has_init ? 1 : 0, n_cus, st);
    else if (keys16_n(P.N))
        launch_walk_t<uint16_t, false>(P, L, keys, final_inv, has_init ? 1 : 0, n_cus, st);
    else
        launch_walk_t<uint32_t, false>(P, L, keys, final_inv, has_init ? 1 : 0, n_cus, st);
    return hipGetLastError();
}

} // namespace pk

// Internal declarations of libpicard (HIP, gfx950).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/picard.h"

namespace pk {

constexpr int WAVE = 64;
constexpr int LOST = PK_LOST;
constexpr int32_t FR_ALL = -1;          // frontier: every run of the SKU is active
constexpr int32_t FR_NONE = 0x7fffffff; // frontier: nothing changed (SKU converged)

// Device view of the problem (pk_problem with the trajectory offsets on the device).
struct Prob {
    int32_t N, K, R, n_traj;
    int64_t total;
    const int32_t *sku, *region, *qty, *x0, *cost;
    const int64_t *traj_off; // device [n_traj+1]
    uint64_t seed;
};

// Control block in device memory: the pass loop runs without host round trips; every
// pass kernel reads `pass`/`done` and the end-of-pass kernel advances them.
constexpr int STAT_SLOTS = 64; // statistics are spread over slots to avoid one hot address
enum { ST_ORDERS = 0, ST_RUNS, ST_CHANGED, ST_BYTES, ST_NEAR_TIES, ST_FLOPS, ST_SCAN_BYTES, ST_N };

// Ctl::error bits set by device-side consistency checks (the validate bits are 1..8).
constexpr int32_t ERR_NO_PROGRESS = 1 << 12; // a walk step could not commit any order
constexpr int32_t ERR_PARTITION = 1 << 4;    // a given partition names a negative process

struct Ctl {
    int32_t pass;        // current pass (1-based)
    int32_t done;        // 1 once a pass changed nothing, 2 when max_passes was reached
    int32_t any_changed; // this pass
    int32_t n_sr, n_seg, n_split, n_split_seg; // setup products
    int32_t error;       // validate: nonzero if an input value was out of range
    int32_t passes_done; // pass count at convergence
    int32_t max_passes;
    uint32_t wg_done;    // workgroups of the current walk launch that have finished
    int32_t n_active;    // runs listed in Plan::active for the current pass
    int32_t n_wide;      // first pass: runs the wave-per-run walk takes (Plan::wlist head)
    int32_t n_lane;      // first pass: runs walked one per lane (Plan::wlist after n_wide)
    int32_t qty_unpacked; // setup: some quantity did not fit the sort key word
    int32_t rq_bad;       // setup: some quantity did not fit Plan::s_rq (no lane walk)
    unsigned long long stat[STAT_SLOTS][ST_N]; // summed on the host
};

// Everything a walk needs to start a run, in one 32-byte record (one load per run).
struct RunDesc {
    int32_t lo, hi; // sorted positions [lo, hi)
    int32_t key;    // trajectory * K + SKU
    int32_t g;      // segment
    int32_t j;      // index of the run in its segment
    int32_t nsr;    // runs in the segment
    int32_t uidx;   // row of u/E (split segments), else -1
    int32_t pad;
};

// Products of the per-call setup (partition and sort), all in the caller's workspace.
struct Plan {
    int32_t B;               // block length
    int32_t n_keys;          // n_traj * K
    int32_t no_frontier;     // 1: every run is re-walked every pass
    int32_t *perm;           // [total] sorted position -> original order index
    int32_t *s_key;          // [total] sorted (trajectory, SKU) key
    int32_t *s_region;       // [total]
    int32_t *s_qty;          // [total]
    int32_t *s_alpha;        // [total] cached action (sorted order)
    int32_t *s_ship;         // [total] units shipped (sorted order)
    int32_t *s_t;            // [total] time index within the trajectory (learned only)
    int32_t *sr_lo;          // [n_sr_max+1] first sorted position of each run
    int32_t *sr_seg;         // [n_sr_max] segment (SKU list) of each run
    int32_t *sr_uidx;        // [n_sr_max] row of u/E for runs of split segments, else -1
    int32_t *seg_key;        // [n_seg_max]
    int32_t *seg_sr0;        // [n_seg_max+1] first run of each segment
    RunDesc *rd;             // [n_sr_max] run descriptors
    int32_t *active;         // [n_split_max] runs to walk in the current pass (after pass 1)
    int32_t *split_list;     // [n_split_max] runs of split segments, in order
    int32_t *split_segs;     // [n_seg_max] split segments
    int32_t *fr[2];          // [n_seg_max] frontier per segment, by pass parity
    int32_t *u;              // [n_split_max][N] cached consumption of each split run
    int32_t *E;              // [n_split_max][N] consumption entering each split run
    float *costT;            // [n_traj][R][N] cost as float, region-major (learned policy)
    void *pos;               // greedy: key table of greedy_keys.h
    uint8_t *pref;           // greedy, N <= 128: preference lists of greedy_keys.h
    int32_t *wlist;          // nullable [n_sr_max] first-pass run list: runs longer than
                             // lane_max in run order, then the others longest first
    int32_t lane_max;        // the longest run the first pass walks one per lane
    int32_t *s_rq;           // nullable [total] region | quantity << rq_rb (lane walk)
    int32_t rq_rb;           // region bits of s_rq
    int32_t pref_lds;        // 1: the lane walk may stage a trajectory's preference lists in LDS
    const int32_t *worker;   // nullable [total] process of each order (original order);
                             // null: blocks of B sorted positions are the processes
    int32_t *ch_prevj;       // [n_sr_max] given partitions: index within its segment of the
                             // previous run of the same process, -1 if none
    int32_t *ch_next;        // [n_sr_max] given partitions: next run of the same process in
                             // the segment, -1 if none
    int32_t *traj_lcp;       // [n_traj] last pass in which the trajectory changed
    int32_t *sink;           // [256] write target of masked-off lanes (contents unused)
    Ctl *ctl;
};

// ---------------------------------------------------------------- wave helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt()
{
    int l = __lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Compiler barrier + LDS ordering point for one wavefront (no hardware cost).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ int wave_incl_sum(int v)
{
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        int o = __shfl_up(v, d, WAVE);
        if (__lane_id() >= d) v += o;
    }
    return v;
}

__device__ __forceinline__ int wave_sum(int v)
{
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, WAVE);
    return v;
}

__device__ __forceinline__ int traj_of(const int64_t *off, int n_traj, int64_t o)
{
    int lo = 0, hi = n_traj; // off[lo] <= o < off[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= o) lo = mid; else hi = mid;
    }
    return lo;
}

// End of a pass (one thread): a pass that changed nothing ends the iteration (Algorithm 1
// returns); otherwise the next pass begins, unless max_passes is reached.
__device__ __forceinline__ void pass_end_body(Ctl *ctl)
{
    if (ctl->done) return;
    if (!ctl->any_changed) {
        ctl->done = 1;
        ctl->passes_done = ctl->pass;
    } else if (ctl->pass >= ctl->max_passes) {
        ctl->done = 2;
        ctl->passes_done = ctl->pass;
    } else {
        ctl->pass += 1;
    }
    ctl->any_changed = 0;
    ctl->n_active = 0;
}

// Called by every workgroup of a walk launch as its last action, with each wave's "some
// run of mine changed" flag: the workgroup raises the pass's change flag once, and the
// workgroup that finishes last (ticket) ends the pass.  Release fence before the ticket,
// acquire fence in the last workgroup, so the other workgroups' flags are visible to it.
__device__ __forceinline__ void walk_finish(Ctl *ctl, bool wave_changed)
{
    __shared__ int32_t s_changed;
    if (threadIdx.x == 0) s_changed = 0;
    __syncthreads();
    if (wave_changed && __lane_id() == 0) s_changed = 1;
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_changed) ctl->any_changed = 1;
        __threadfence();
        const unsigned prev = atomicAdd(&ctl->wg_done, 1u);
        if (prev == gridDim.x - 1) {
            __threadfence();
            ctl->wg_done = 0;
            pass_end_body(ctl);
            __threadfence();
        }
    }
}

// Coefficients of one Adam step, each rounded once to float32 from its double value.
struct AdamCoef {
    float lr, b1, b2, omb1, omb2, bc1, bc2, eps, dir;
};

// ---------------------------------------------------------------- host launchers
// All return hipSuccess or the first HIP error.  `st` is the stream.

// First pass of the greedy walk (N <= 128, block partitions): runs up to Plan::lane_max
// orders (at most LANE_MAX_LEN) are walked one per lane (walk_lane.hip), longer ones a wave
// per run.
constexpr int LANE_MAX_LEN = 510;
int lane_max_for(int64_t total, int N, int R, int n_cus);
constexpr int PREF_MAX_N = 128; // the greedy preference lists (greedy_keys.h) exist up to here
size_t walk_lane_lds(int N, int R);
bool pref_in_lds(int N, int R);
int region_bits(int R);
hipError_t launch_walk_greedy_lane(const Prob &P, const Plan &L, int32_t *final_inv,
                                   bool has_init, int64_t n_list, hipStream_t st);
hipError_t scan_i64(int64_t *data, int64_t n, bool inclusive, void *tmp, hipStream_t st);
hipError_t scan_i64_to(const int64_t *src, int64_t *dst, int64_t n, bool inclusive, void *tmp,
                       hipStream_t st); // out of place
size_t scan_tmp_bytes(int64_t n);
hipError_t scan_i32_excl(int32_t *data, int64_t n, void *tmp, hipStream_t st);

hipError_t radix_sort_pairs(int32_t *keys, int32_t *vals, int32_t *keys_alt,
                            int32_t *vals_alt, int64_t n, int key_bits, void *tmp,
                            hipStream_t st, bool *result_in_alt);
size_t radix_tmp_bytes(int64_t n);
// Stable sort by bits [0, key_bits) within each segment [seg_off[s], seg_off[s+1]) (device
// offsets, n_seg segments covering [0, n)); tmp of radix_tmp_bytes(n, n_seg).
hipError_t radix_sort_pairs_seg(int32_t *keys, int32_t *vals, int32_t *keys_alt,
                                int32_t *vals_alt, int64_t n, int key_bits,
                                const int64_t *seg_off, int n_seg, void *tmp, hipStream_t st,
                                bool *result_in_alt);
size_t radix_tmp_bytes(int64_t n, int n_seg);
int radix_passes(int key_bits);
// out_a[perm[p]] = a[p], out_b[perm[p]] = b[p] (b, out_b nullable) for a permutation within
// each segment; segments of at most 2^20 elements and a in [-1, 4094] (unpermute_fits).
// Four int32 arrays of n and radix_tmp_bytes(n, n_seg) of tmp.
bool unpermute_fits(int64_t longest_segment, int32_t a_max);
hipError_t unpermute_seg(const int32_t *perm, const int32_t *a, const int32_t *b, int64_t n,
                         const int64_t *seg_off, int n_seg, int32_t *out_a, int32_t *out_b,
                         int32_t *k0, int32_t *v0, int32_t *k1, int32_t *v1, void *tmp,
                         hipStream_t st);
hipError_t launch_unpermute(const Prob &P, const Plan &L, int32_t *actions, int32_t *shipped,
                            hipStream_t st);

// ---------------------------------------------------------------- OWMR inventory control
// (owmr.hip: one central warehouse and N retailers, one process per retailer)
struct OwmrDev {
    int32_t N;
    int64_t T;
    const int32_t *retailer, *demand, *s_ret, *S_ret, *cap, *x_init;
    int64_t s0, S0, x0_init;
};

struct OwmrCtl {
    int32_t pass, done, passes_done, max_passes;
    int32_t error;
    unsigned long long changed;          // steps whose action changed in the current pass
    unsigned long long changed_log[8];   // the last eight passes' counts, by pass % 8
};

size_t owmr_radix_tmp(int64_t T);
hipError_t owmr_launch_setup(const OwmrDev &P, int32_t *keys, int32_t *keys_alt, int32_t *vals,
                             int32_t *vals_alt, void *rtmp, int32_t *cnt, void *stmp,
                             int32_t *sd, int32_t *err, int32_t **perm, hipStream_t st);
hipError_t owmr_launch_init(const OwmrDev &P, const int32_t *iq, const int32_t *ir, int64_t *V,
                            OwmrCtl *ctl, int32_t max_passes, hipStream_t st);
hipError_t owmr_launch_pass(const OwmrDev &P, OwmrCtl *ctl, const int32_t *perm, const int32_t *sd,
                            const int32_t *seg, int64_t *V, int64_t *S, int64_t *rq, void *stmp,
                            int64_t *fx0v, int32_t *fx, int64_t *caches, int64_t *sink,
                            hipStream_t st); // sink: [64] stores of lanes without a retailer
hipError_t owmr_launch_unpack(const OwmrDev &P, const int64_t *V, int32_t *q, int32_t *r,
                              hipStream_t st);
hipError_t owmr_launch_serial(const OwmrDev &P, int32_t *q, int32_t *r, int64_t *fx0, int32_t *fx,
                              unsigned long long *resets, hipStream_t st);

// ---------------------------------------------------------------- node capacity
// (capacity.hip: Picard with the FO state (x, c) of Section 3, time-block processes)
constexpr int CAP_NPAD = 128; // warehouses per row: two per lane
constexpr int CAP_MAX_B = 255;
constexpr int CAP_PIECE = 512; // positions of the SKU-sorted list per entry wave
constexpr int CAP_GROUP = 4;   // passes launched per host check of the change counts
constexpr uint32_t CAP_NONE = 0xffffffffu;

// error bits of CapCtl::error
constexpr int32_t CAP_ERR_QTY = 1, CAP_ERR_SKU = 2, CAP_ERR_REGION = 4, CAP_ERR_X0 = 8,
                  CAP_ERR_CAP = 16, CAP_ERR_COST = 32, CAP_ERR_INIT = 64, CAP_ERR_BID = 128;
// Capacity policies (the walk's template argument)
constexpr int CAP_GREEDY = 0, CAP_GAMMA = 1, CAP_BID = 2;

struct CapCtl {
    int32_t error;
    int32_t pass;      // current pass, from 1
    int32_t first_blk; // first block with a change in the current pass
    int32_t frontier;  // blocks <= frontier are not walked in the current pass
    int32_t n_pieces;
    int32_t max_distinct; // the most distinct SKUs in one block
};

struct CapPlan {
    int32_t T, N, K, R, B, nblk;
    int32_t gnum, gden;  // policy: 0 = greedy, else capacity-dependent, gamma = gnum / gden
    int32_t glow;        // capacity-dependent: 0 = price relative to the most capacity left,
                         // else only nodes with less than glow left pay a price
    int32_t dmax;        // stock rows per block in the walk's LDS (CapCtl::max_distinct)
    int32_t pol;         // CAP_GREEDY, CAP_GAMMA or CAP_BID
    const int32_t *bid_inv; // [K][N] bid prices of stock, nullable (CAP_BID)
    const int32_t *bid_cap; // [N] bid prices of capacity, nullable (CAP_BID)
    int64_t max_pieces;
    const int32_t *sku, *region, *qty, *x0, *cost, *cap0;
    int32_t *alpha;      // [T] cache, time order (the caller's actions buffer)
    int32_t *perm;       // [T] SKU-sorted position -> time index
    int32_t *seg_off;    // [K+1]
    int32_t *slot;       // [T] rank of its SKU among the block's distinct SKUs (LDS row)
    int32_t *first;      // [T] 1 for the first order of each (block, SKU)
    int32_t *sid;        // [T] row of X for the first order of each (block, SKU)
    int32_t *srow;       // [T] sorted position -> row of X it starts, or -1
    int32_t *piece_off;  // [K+1] first piece of each SKU
    int4 *piece;         // [max_pieces] SKU, first and end sorted position, several pieces
    int32_t *pc;         // [max_pieces][CAP_NPAD] action counts, then their scan
    int32_t *H;          // [N][nblk] passing cached actions per (node, block)
    int32_t *capE;       // [N][nblk] capacity at each block's start
    uint32_t *keyT;      // [R][CAP_NPAD] (cost << 8) | w (greedy), rank (capacity-dependent)
                         // or cost + bid_cap[w] (bid prices); all-ones past N
    uint8_t *X;          // [T][CAP_NPAD] stock rows of the (block, SKU) pairs
    uint8_t *P;          // [T] 1 if the order's cached action passes its stock test
    int32_t *skuchg;     // [K] last pass in which an order of the SKU changed its action
    int32_t *chg;        // [CAP_GROUP] orders whose action changed, per pass of a group
    CapCtl *ctl;
};

size_t cap_walk_lds(int B, int D);
hipError_t cap_check(CapPlan &L, const int32_t *init, hipStream_t st);
hipError_t cap_setup(CapPlan &L, int32_t *keys, int32_t *vals, int32_t *keys_alt,
                     int32_t *vals_alt, int32_t *first, void *tmp, hipStream_t st);
hipError_t cap_pass(const CapPlan &L, bool first, hipStream_t st);
hipError_t cap_finish(const CapPlan &L, int32_t *final_inv, int32_t *final_cap, int32_t *used,
                      hipStream_t st);
hipError_t cap_serial_setup(CapPlan &L, hipStream_t st);
hipError_t cap_serial(const CapPlan &L, int32_t *state, int32_t *actions, hipStream_t st);

} // namespace pk

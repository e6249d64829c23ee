// C-ABI entry points of libpicard (declared in include/picard.h).
#include <hip/hip_runtime.h>

#include <dlfcn.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <map>
#include <mutex>
#include <vector>

#include "pk_internal.h"

namespace pk {
// setup.hip
hipError_t setup_ctl(Plan &L, int n_traj, int max_passes, hipStream_t st);
hipError_t setup_plan(const Prob &P, Plan &L, const int32_t *init_cache, int validate,
                      bool want_t, int32_t n_seg_max, void *scratch, hipStream_t st);
size_t setup_scratch_bytes(int64_t n, int n_traj);
hipError_t setup_pos(const Prob &P, void *pos, uint8_t *pref, hipStream_t st);
size_t pos_bytes(int N, int R, int n_traj);
size_t pref_bytes(int N, int R, int n_traj);
// pass.hip
hipError_t launch_scan_entry(const Prob &P, const Plan &L, int n_seg_max, bool skip_first,
                             hipStream_t st);
hipError_t launch_pass_end(const Plan &L, hipStream_t st);
hipError_t launch_consume(const Prob &P, const Plan &L, int64_t n_split_max, hipStream_t st);
hipError_t unpermute_results(const Prob &P, const Plan &L, int32_t *actions, int32_t *shipped,
                             void *scratch, bool tiles, hipStream_t st);
// walk_chain.hip
hipError_t launch_walk_chain_greedy(const Prob &P, const Plan &L, int32_t *final_inv,
                                    bool has_init, int n_cus, hipStream_t st);
// walk_greedy.hip
size_t walk_greedy_lds(int N, int R);
hipError_t launch_walk_greedy(const Prob &P, const Plan &L, const void *keys, int32_t *final_inv,
                              bool has_init, int n_cus, hipStream_t st);
// greedy.hip
hipError_t launch_serial_greedy(const Prob &P, const void *pos, int32_t *state, int32_t *actions,
                                int32_t *shipped, hipStream_t st);
// mlp.hip
size_t costT_bytes(int N, int R, int n_traj);
hipError_t setup_costT(const Prob &P, const float *params, float *costT, hipStream_t st);
size_t walk_mlp_lds(int N);
hipError_t launch_walk_mlp(const Prob &P, const Plan &L, const float *params, int layers,
                           const float *costT, int32_t *final_inv, bool has_init, int n_cus,
                           int waves, hipStream_t st);
hipError_t launch_serial_mlp(const Prob &P, const float *params, int layers, const float *costT,
                             int32_t *state, int32_t *actions, int32_t *shipped, hipStream_t st);
hipError_t launch_scores(const Prob &P, const float *params, int layers, const float *costT,
                         int b, int r, const int32_t *xrow, float *out, hipStream_t st);
// grad.hip
size_t grad_lds(int N, int layers);
int grad_wg_per_cu(int N);
size_t grad_part_bytes(int n_wg, int R, int layers);
hipError_t launch_grad(const Prob &P, const Plan &L, const float *params, int layers,
                       const float *costT, const float *adv, float *logp_sorted, double *part,
                       int n_wg, float *grad, double *objective_dev, float *logp_out,
                       hipStream_t st);
// train.hip
size_t advantages_ws_bytes(int64_t total, int n_traj);
hipError_t launch_advantages(const int64_t *offs_dev, int n_traj, int N, int R, int64_t total,
                             const int32_t *region, const int32_t *actions,
                             const int32_t *shipped, const int32_t *cost, int32_t revenue,
                             int64_t rlim, int64_t *rew, unsigned long long *wsum, int32_t *err,
                             void *scan_tmp, float *adv, int64_t *ret, hipStream_t st);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, int64_t n,
                       const AdamCoef &c, hipStream_t st);
} // namespace pk

using namespace pk;

// Scratch of pk_picard_simulate_noalloc: the workspace of one simulation, held by every
// device the library runs on until the process ends.  Host code never passes this name to
// a kernel or a copy (on the host it is only a stand-in); it uses the device address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[PK_NOALLOC_SCRATCH_BYTES];

namespace {

// Message of the last failed call on this thread (a fixed buffer: reporting an error
// allocates nothing).
thread_local char g_err[512];

pk_status fail(pk_status s, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

// Device address of `scratch` per device, resolved once per device with that device
// current (each device holds its own copy of the array at its own address).
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

pk_status scratch_on_current_device(void **out)
{
    int dev = -1;
    const hipError_t ge = hipGetDevice(&dev);
    if (ge != hipSuccess) return fail(PK_ERR_HIP, "hipGetDevice failed: %s", hipGetErrorString(ge));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(PK_ERR_UNSUPPORTED, "device %d: the static scratch serves devices 0..%d",
                    dev, NOALLOC_MAX_DEVICES - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(PK_ERR_HIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return PK_OK;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t _e = (expr);                                                              \
        if (_e != hipSuccess)                                                                \
            return fail(PK_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(_e));          \
    } while (0)

constexpr int DEFAULT_BLOCK_GREEDY = 1024;
constexpr int DEFAULT_BLOCK_MLP = 1024;
constexpr int GRAD_BLOCK = 1024;  // run length of the gradient's state reconstruction
constexpr int GRAD_MAX_WG = 512;  // workgroups (and FP64 partial sets) of the gradient
constexpr int MIN_AUTOTUNE_BLOCK = 64;

struct Dims {
    int32_t N, K, R, n_traj;
    int64_t total, max_T, n_keys;
};

pk_status check_problem(const pk_problem *pr, Dims *d)
{
    if (!pr) return fail(PK_ERR_INVALID_ARG, "problem is NULL");
    if (pr->n_warehouses < 1 || pr->n_skus < 1 || pr->n_regions < 1 || pr->n_traj < 1)
        return fail(PK_ERR_SHAPE, "dimensions must be >= 1 (N=%d K=%d R=%d n_traj=%d)",
                    pr->n_warehouses, pr->n_skus, pr->n_regions, pr->n_traj);
    if (pr->n_warehouses > PK_MAX_WAREHOUSES)
        return fail(PK_ERR_SHAPE, "N=%d exceeds %d", pr->n_warehouses, PK_MAX_WAREHOUSES);
    if (pr->n_regions > PK_MAX_REGIONS)
        return fail(PK_ERR_SHAPE, "R=%d exceeds %d", pr->n_regions, PK_MAX_REGIONS);
    if (!pr->traj_offsets) return fail(PK_ERR_INVALID_ARG, "traj_offsets is NULL");
    if (pr->traj_offsets[0] != 0) return fail(PK_ERR_SHAPE, "traj_offsets[0] must be 0");
    int64_t maxT = 0;
    for (int b = 0; b < pr->n_traj; ++b) {
        const int64_t len = pr->traj_offsets[b + 1] - pr->traj_offsets[b];
        if (len < 0) return fail(PK_ERR_SHAPE, "traj_offsets must be nondecreasing");
        maxT = std::max(maxT, len);
    }
    const int64_t total = pr->traj_offsets[pr->n_traj];
    if (total >= (1ll << 31) - 1) return fail(PK_ERR_SHAPE, "total orders must be < 2^31");
    const int64_t n_keys = (int64_t)pr->n_traj * pr->n_skus;
    if (n_keys >= (1ll << 31) - 1) return fail(PK_ERR_SHAPE, "n_traj*K must be < 2^31");
    if (total > 0 && (!pr->sku || !pr->region || !pr->qty))
        return fail(PK_ERR_INVALID_ARG, "order arrays are NULL");
    if (!pr->init_inv || !pr->cost) return fail(PK_ERR_INVALID_ARG, "init_inv/cost is NULL");
    d->N = pr->n_warehouses;
    d->K = pr->n_skus;
    d->R = pr->n_regions;
    d->n_traj = pr->n_traj;
    d->total = total;
    d->max_T = maxT;
    d->n_keys = n_keys;
    return PK_OK;
}

pk_status check_policy(const pk_policy *po)
{
    if (!po) return fail(PK_ERR_INVALID_ARG, "policy is NULL");
    if (po->kind == PK_POLICY_GREEDY) return PK_OK;
    if (po->kind != PK_POLICY_MLP) return fail(PK_ERR_INVALID_ARG, "unknown policy kind %d", po->kind);
    if (!po->params) return fail(PK_ERR_INVALID_ARG, "MLP params are NULL");
    if (po->hidden != 64 || po->emb_dim != 16 ||
        (po->n_hidden_layers != 1 && po->n_hidden_layers != 2))
        return fail(PK_ERR_UNSUPPORTED, "MLP must have hidden=64, emb_dim=16, 1 or 2 layers");
    return PK_OK;
}

// ---------------------------------------------------------------- workspace layout
struct Carver {
    char *base;
    size_t off = 0;
    template <typename T>
    T *take(int64_t count)
    {
        T *p = base ? (T *)(base + off) : nullptr;
        off += ((size_t)std::max<int64_t>(count, 1) * sizeof(T) + 255) & ~(size_t)255;
        return p;
    }
};

struct Sizes {
    int64_t n_sr_max, n_seg_max, n_split_max;
};

Sizes plan_sizes(const Dims &d, int B)
{
    Sizes s;
    const int64_t nblocks = (d.total + B - 1) / B;
    s.n_seg_max = std::max<int64_t>(1, std::min<int64_t>(d.total, d.n_keys));
    s.n_sr_max = nblocks + s.n_seg_max + 1;
    s.n_split_max = std::max<int64_t>(1, std::min<int64_t>(s.n_sr_max, 2 * nblocks));
    return s;
}

// Carves the Picard plan (or just measures it when base == nullptr).
void carve_plan(Carver &c, const Dims &d, const pk_policy *po, int B, Plan *L,
                int64_t **traj_off, void **setup_scratch)
{
    const Sizes s = plan_sizes(d, B);
    Plan p = {};
    p.B = B;
    p.n_keys = (int32_t)d.n_keys;
    p.ctl = c.take<Ctl>(1);
    *traj_off = c.take<int64_t>(d.n_traj + 1);
    p.traj_lcp = c.take<int32_t>(d.n_traj);
    p.sink = c.take<int32_t>(4 * 64); // four 64-lane rows of dummy stores
    p.perm = c.take<int32_t>(d.total);
    p.s_key = c.take<int32_t>(d.total);
    p.s_region = c.take<int32_t>(d.total);
    p.s_qty = c.take<int32_t>(d.total);
    p.s_alpha = c.take<int32_t>(d.total);
    p.s_ship = c.take<int32_t>(d.total);
    p.s_t = po->kind == PK_POLICY_MLP ? c.take<int32_t>(d.total) : nullptr;
    p.sr_lo = c.take<int32_t>(s.n_sr_max + 1);
    p.sr_seg = c.take<int32_t>(s.n_sr_max);
    p.sr_uidx = c.take<int32_t>(s.n_sr_max);
    p.ch_prevj = c.take<int32_t>(s.n_sr_max);
    p.ch_next = c.take<int32_t>(s.n_sr_max);
    p.seg_key = c.take<int32_t>(s.n_seg_max);
    p.seg_sr0 = c.take<int32_t>(s.n_seg_max + 1);
    p.split_segs = c.take<int32_t>(s.n_seg_max);
    p.fr[0] = c.take<int32_t>(s.n_seg_max);
    p.fr[1] = c.take<int32_t>(s.n_seg_max);
    p.split_list = c.take<int32_t>(s.n_split_max);
    p.rd = c.take<RunDesc>(s.n_sr_max);
    p.active = c.take<int32_t>(s.n_split_max);
    p.u = c.take<int32_t>(s.n_split_max * d.N);
    p.E = c.take<int32_t>(s.n_split_max * d.N);
    if (po->kind == PK_POLICY_MLP)
        p.costT = c.take<float>((int64_t)costT_bytes(d.N, d.R, d.n_traj) / 4);
    else
        p.pos = c.take<char>((int64_t)pos_bytes(d.N, d.R, d.n_traj));
    if (po->kind != PK_POLICY_MLP && d.N <= PREF_MAX_N) { // the first pass's lane walk
        p.pref = c.take<uint8_t>((int64_t)pref_bytes(d.N, d.R, d.n_traj));
        p.wlist = c.take<int32_t>(s.n_sr_max);
        p.s_rq = c.take<int32_t>(d.total);
        p.rq_rb = region_bits(d.R);
        p.pref_lds = pref_in_lds(d.N, d.R) ? 1 : 0;
    }
    *setup_scratch = c.take<char>((int64_t)setup_scratch_bytes(d.total, d.n_traj));
    if (L) *L = p;
}

size_t serial_bytes(const Dims &d)
{
    Carver c{nullptr};
    c.take<int64_t>(d.n_traj + 1);
    c.take<char>((int64_t)std::max(pos_bytes(d.N, d.R, d.n_traj), costT_bytes(d.N, d.R, d.n_traj)));
    c.take<int32_t>((int64_t)d.n_traj * d.K * d.N);
    return c.off + 256;
}

size_t picard_bytes(const Dims &d, const pk_policy *po, int B)
{
    Carver c{nullptr};
    int64_t *to;
    void *ss;
    carve_plan(c, d, po, B, nullptr, &to, &ss);
    return c.off + 256;
}

size_t grad_bytes(const Dims &d, const pk_policy *po)
{
    Carver c{nullptr};
    int64_t *to;
    void *ss;
    carve_plan(c, d, po, GRAD_BLOCK, nullptr, &to, &ss);
    c.take<float>(d.total);
    c.take<char>((int64_t)grad_part_bytes(GRAD_MAX_WG, d.R, po->n_hidden_layers));
    c.take<double>(1);
    return c.off + 256;
}

char *align_ws(void *ws) { return (char *)(((uintptr_t)ws + 255) & ~(uintptr_t)255); }

Prob make_prob(const pk_problem *pr, const Dims &d, const int64_t *traj_off_dev)
{
    Prob P;
    P.N = d.N;
    P.K = d.K;
    P.R = d.R;
    P.n_traj = d.n_traj;
    P.total = d.total;
    P.sku = pr->sku;
    P.region = pr->region;
    P.qty = pr->qty;
    P.x0 = pr->init_inv;
    P.cost = pr->cost;
    P.traj_off = traj_off_dev;
    P.seed = pr->rng_seed;
    return P;
}

struct PinnedCtl {
    Ctl *h = nullptr;
    ~PinnedCtl()
    {
        if (h) (void)hipHostFree(h);
    }
    Ctl *get()
    {
        if (!h && hipHostMalloc((void **)&h, sizeof(Ctl), hipHostMallocDefault) != hipSuccess)
            h = nullptr;
        return h;
    }
};
thread_local PinnedCtl g_pinned;

int num_cus()
{
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
        return 256;
    return n;
}

// ---------------------------------------------------------------- captured pass graphs
// The instantiated graph of U passes is kept per thread and reused while every kernel
// argument is unchanged (same problem, plan and output buffers).
struct GraphKey {
    unsigned char bytes[sizeof(Prob) + sizeof(Plan) + sizeof(pk_policy) + 80];
    // setup: the graph also holds the per-call setup, which depends on the remaining
    // arguments (the warm-start cache, validation, the pass limit seeded in the control
    // block)
    void set(const Prob &P, const Plan &L, const pk_policy *po, const int32_t *fin, bool hi,
             int grid, int U, int nseg, bool timing, bool setup = false,
             const int32_t *init_cache = nullptr, int validate = 0, int max_passes = 0)
    {
        memset(bytes, 0, sizeof bytes);
        size_t o = 0;
        memcpy(bytes + o, &P, sizeof P); o += sizeof P;
        memcpy(bytes + o, &L, sizeof L); o += sizeof L;
        memcpy(bytes + o, po, sizeof *po); o += sizeof *po;
        const int64_t extra[10] = {(int64_t)(uintptr_t)fin, hi, grid, U, nseg, timing, setup,
                                   (int64_t)(uintptr_t)init_cache, validate, max_passes};
        static_assert(sizeof(extra) + sizeof(P) + sizeof(L) + sizeof(pk_policy) <= sizeof(bytes),
                      "graph key too small");
        memcpy(bytes + o, extra, sizeof extra);
    }
    bool operator==(const GraphKey &k) const { return memcmp(bytes, k.bytes, sizeof bytes) == 0; }
};

// When timing is requested the graph also holds an event pair around every walk (event
// record nodes added to the graph being captured); every replay records them again.
pk_status record_in_capture(hipStream_t s, hipEvent_t e)
{
    hipStreamCaptureStatus cs;
    unsigned long long id = 0;
    hipGraph_t g = nullptr;
    const hipGraphNode_t *deps = nullptr;
    size_t nd = 0;
    HIP_TRY(hipStreamGetCaptureInfo_v2(s, &cs, &id, &g, &deps, &nd));
    if (cs != hipStreamCaptureStatusActive || !g) return fail(PK_ERR_HIP, "stream is not capturing");
    hipGraphNode_t node = nullptr;
    HIP_TRY(hipGraphAddEventRecordNode(&node, g, deps, nd, e));
    HIP_TRY(hipStreamUpdateCaptureDependencies(s, &node, 1, hipStreamSetCaptureDependencies));
    return PK_OK;
}

// Captured graphs, a few per thread (least recently used dropped first), so that calls
// alternating between problems or block lengths (the autotuner) keep theirs.
struct GraphEntry {
    bool valid = false;
    int device = -1;
    uint64_t used = 0;
    GraphKey key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipEvent_t> evs;
    void clear()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (hipEvent_t e : evs) (void)hipEventDestroy(e);
        evs.clear();
        exec = nullptr;
        graph = nullptr;
        valid = false;
    }
};

struct GraphCache {
    static constexpr int SLOTS = 32; // the autotuner cycles through 13 block lengths x 2 graphs
    GraphEntry slot[SLOTS];
    uint64_t tick = 0;
    hipStream_t cap = nullptr;
    int cap_device = -1;
    ~GraphCache()
    {
        for (GraphEntry &e : slot) e.clear();
    }
    // The entry for key k, captured by enqueue(stream, entry) on a miss; n_events events are
    // created for the capture to record.
    template <typename F> pk_status get(const GraphKey &k, int n_events, F enqueue,
                                        GraphEntry **out)
    {
        int dev = 0;
        HIP_TRY(hipGetDevice(&dev));
        ++tick;
        GraphEntry *victim = &slot[0];
        for (GraphEntry &e : slot) {
            if (e.valid && e.device == dev && e.key == k) {
                e.used = tick;
                *out = &e;
                return PK_OK;
            }
            if (!e.valid) victim = &e;
            else if (victim->valid && e.used < victim->used) victim = &e;
        }
        victim->clear();
        if (cap && dev != cap_device) {
            (void)hipStreamDestroy(cap);
            cap = nullptr;
        }
        if (!cap) {
            HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
            cap_device = dev;
        }
        for (int i = 0; i < n_events; ++i) {
            hipEvent_t e = nullptr;
            HIP_TRY(hipEventCreate(&e));
            victim->evs.push_back(e);
        }
        HIP_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        pk_status e = enqueue(cap, *victim);
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(cap, &g);
        if (e != PK_OK) {
            if (g) (void)hipGraphDestroy(g);
            victim->clear();
            return e;
        }
        if (ce != hipSuccess) {
            victim->clear();
            return fail(PK_ERR_HIP, "graph capture failed: %s", hipGetErrorString(ce));
        }
        victim->graph = g;
        const hipError_t ie = hipGraphInstantiate(&victim->exec, g, nullptr, nullptr, 0);
        if (ie != hipSuccess) {
            victim->clear();
            return fail(PK_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(ie));
        }
        victim->key = k;
        victim->device = dev;
        victim->used = tick;
        victim->valid = true;
        *out = victim;
        return PK_OK;
    }
};
thread_local GraphCache g_graph;

// Passes the last call on the same problem and plan needed: the next call captures that
// many passes in its graph, so that a repeated simulation runs as one replay with no
// trailing empty passes.  Convergence is still decided on the device; a call that needs
// more passes replays the graph again.
struct LastPasses {
    bool valid = false;
    GraphKey key; // with U = 0
    int passes = 0;
};
thread_local LastPasses g_last_passes;

// noalloc: create nothing (no captured graph, no events, no pinned control block, no host
// heap buffer); the passes are enqueued directly and the control block is read into a
// stack copy.
// abort_ms > 0 (the autotuner): give up, with PK_ERR_NOT_CONVERGED, once the call has
// taken longer than that (checked whenever the host reads the control block).
pk_status picard_run(const pk_problem *problem, const Dims &d, const pk_policy *policy,
                     const pk_picard_opts &o, int B, void *ws, size_t ws_bytes,
                     int32_t *actions, int32_t *shipped, int32_t *final_inv, pk_stats *stats,
                     hipStream_t stream, bool noalloc = false, double abort_ms = 0.0)
{
    const auto t_call = std::chrono::steady_clock::now();
    const int waves = o.walk_waves == 8 ? 8 : 4;
    const int64_t mp64 = o.max_passes > 0 ? o.max_passes : d.max_T + 1;
    const int max_passes = (int)std::min<int64_t>(mp64, 0x7ffffff0);
    if (!ws || ws_bytes < picard_bytes(d, policy, B))
        return fail(PK_ERR_WORKSPACE, "workspace too small: need %zu bytes, got %zu",
                    picard_bytes(d, policy, B), ws_bytes);
    if (policy->kind == PK_POLICY_GREEDY && walk_greedy_lds(d.N, d.R) > 65536)
        return fail(PK_ERR_SHAPE, "N=%d, R=%d need more LDS than a workgroup has", d.N, d.R);
    hipStream_t st = stream;
    Carver c{align_ws(ws)};
    Plan L;
    int64_t *to;
    void *setup_scr;
    carve_plan(c, d, policy, B, &L, &to, &setup_scr);
    L.no_frontier = o.use_frontier ? 0 : 1;
    L.worker = o.partition;
    L.lane_max = o.lane_max > 0 ? std::min(o.lane_max, LANE_MAX_LEN)
                                : (o.lane_max < 0 ? 0 : lane_max_for(d.total, d.N, d.R, num_cus()));
    if (L.worker || L.lane_max == 0) { // given partitions walk chains; or no lane walk
        L.wlist = nullptr;
        L.s_rq = nullptr;
    }
    const bool lanes = L.wlist != nullptr;
    const Sizes sz = plan_sizes(d, B);
    HIP_TRY(hipMemcpyAsync(to, problem->traj_offsets, (d.n_traj + 1) * sizeof(int64_t),
                           hipMemcpyHostToDevice, st));
    Prob P = make_prob(problem, d, to);
    const bool has_init = o.init_cache != nullptr;
    // the per-call setup: control block, sort and tables, policy tables, warm start, final
    // inventory initialised to x0 (enqueued directly or captured with the first passes)
    auto enqueue_setup = [&](hipStream_t s2) -> pk_status {
        HIP_TRY(setup_ctl(L, d.n_traj, max_passes, s2));
        if (d.total > 0) {
            const bool mlp = policy->kind == PK_POLICY_MLP;
            HIP_TRY(setup_plan(P, L, o.init_cache, o.validate, mlp, (int32_t)sz.n_seg_max,
                               setup_scr, s2));
            if (mlp)
                HIP_TRY(setup_costT(P, policy->params, L.costT, s2));
            else
                HIP_TRY(setup_pos(P, L.pos, L.pref, s2));
            if (has_init) HIP_TRY(launch_consume(P, L, sz.n_split_max, s2));
        }
        if (final_inv)
            HIP_TRY(hipMemcpyAsync(final_inv, problem->init_inv,
                                   (size_t)d.n_traj * d.K * d.N * 4, hipMemcpyDeviceToDevice, s2));
        return PK_OK;
    };
    Ctl ctl_copy;
    Ctl *hc = noalloc ? &ctl_copy : g_pinned.get();
    if (!hc) return fail(PK_ERR_HIP, "pinned host allocation failed");
    const int grid = num_cus(); // the walk sizes its grid from the CU count
    const bool timing = stats && stats->timing && !noalloc;
    int U = o.graph_unroll > 0 ? o.graph_unroll : 8;
    const int gridw = grid * 16 + waves; // the walks' launch shape, part of every graph key
    GraphKey key0; // this call's problem and plan, without the unroll
    key0.set(P, L, policy, final_inv, has_init, gridw, 0, (int)sz.n_seg_max, timing);
    if (o.graph_unroll <= 0 && g_last_passes.valid && g_last_passes.key == key0 &&
        g_last_passes.passes >= 2 && g_last_passes.passes <= 64)
        U = g_last_passes.passes;
    std::vector<hipEvent_t> evs;
    int launched = 0;
    int done = 0;
    if (d.total == 0) {
        done = 1;
    }
    // one pass = entry scan + walk (the walk's last workgroup ends the pass); the kernels
    // return at once after convergence, so U passes are enqueued per host check.
    // Events around the walk: none (ge == nullptr, !with_events), created here, or the
    // captured graph's pair ge[0], ge[1] recorded as graph nodes.
    // pass1: this is the call's first pass (the greedy lane walk runs before the walk)
    auto enqueue_pass = [&](hipStream_t s2, bool with_events, hipEvent_t *ge,
                            bool pass1) -> pk_status {
        hipEvent_t es = nullptr, e0 = nullptr, e1 = nullptr;
        if (ge) {
            const pk_status r = record_in_capture(s2, ge[0]);
            if (r != PK_OK) return r;
        } else if (with_events) {
            HIP_TRY(hipEventCreate(&es));
            HIP_TRY(hipEventCreate(&e0));
            HIP_TRY(hipEventCreate(&e1));
            HIP_TRY(hipEventRecord(es, s2));
        }
        HIP_TRY(launch_scan_entry(P, L, (int)sz.n_seg_max, !has_init, s2));
        if (ge) {
            const pk_status r = record_in_capture(s2, ge[1]);
            if (r != PK_OK) return r;
        } else if (with_events) {
            HIP_TRY(hipEventRecord(e0, s2));
        }
        if (policy->kind == PK_POLICY_MLP)
            HIP_TRY(launch_walk_mlp(P, L, policy->params, policy->n_hidden_layers, L.costT,
                                    final_inv, has_init, num_cus(), waves, s2));
        else if (L.worker)
            HIP_TRY(launch_walk_chain_greedy(P, L, final_inv, has_init, grid, s2));
        else {
            if (lanes && pass1)
                HIP_TRY(launch_walk_greedy_lane(P, L, final_inv, has_init,
                                                std::min<int64_t>(d.total, sz.n_sr_max), s2));
            HIP_TRY(launch_walk_greedy(P, L, L.pos, final_inv, has_init, grid, s2));
        }
        if (ge) {
            const pk_status r = record_in_capture(s2, ge[2]);
            if (r != PK_OK) return r;
        } else if (with_events) {
            HIP_TRY(hipEventRecord(e1, s2));
            evs.push_back(es);
            evs.push_back(e0);
            evs.push_back(e1);
        }
        return PK_OK;
    };
    // graphs: the setup with the first U passes, and U further passes, each captured once
    // and replayed
    GraphEntry *g_first = nullptr, *g_more = nullptr;
    double graph_walk_ms = 0.0, graph_scan_ms = 0.0;
    int64_t graph_walks = 0;
    if (!done && !noalloc && U > 1 && max_passes >= U) {
        for (int with_setup = 1; with_setup >= 0; --with_setup) {
            GraphKey key;
            key.set(P, L, policy, final_inv, has_init, gridw, U, (int)sz.n_seg_max, timing,
                    with_setup != 0, o.init_cache, o.validate, max_passes);
            pk_status gs = g_graph.get(key, timing ? 3 * U : 0,
                                       [&](hipStream_t cs, GraphEntry &ge) -> pk_status {
                if (with_setup) {
                    pk_status e = enqueue_setup(cs);
                    if (e != PK_OK) return e;
                }
                for (int i = 0; i < U; ++i) {
                    pk_status e = enqueue_pass(cs, false, timing ? &ge.evs[3 * i] : nullptr,
                                               with_setup && i == 0);
                    if (e != PK_OK) return e;
                }
                return PK_OK;
            }, with_setup ? &g_first : &g_more);
            if (gs != PK_OK) return gs;
        }
    }
    if (!g_first) {
        const pk_status e = enqueue_setup(st);
        if (e != PK_OK) return e;
    }
    bool first = true;
    while (!done && launched < max_passes) {
        const int u = std::min(U, max_passes - launched);
        GraphEntry *ge = u == U ? (first ? g_first : g_more) : nullptr;
        if (ge) {
            HIP_TRY(hipGraphLaunch(ge->exec, st));
        } else {
            for (int i = 0; i < u; ++i) {
                pk_status e = enqueue_pass(st, timing, nullptr, launched == 0 && i == 0);
                if (e != PK_OK) return e;
            }
        }
        first = false;
        launched += u;
        HIP_TRY(hipMemcpyAsync(hc, L.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (ge && timing) {
            for (int i = 0; i < U; ++i) {
                float ms = 0.f, sms = 0.f;
                HIP_TRY(hipEventElapsedTime(&sms, ge->evs[3 * i], ge->evs[3 * i + 1]));
                HIP_TRY(hipEventElapsedTime(&ms, ge->evs[3 * i + 1], ge->evs[3 * i + 2]));
                graph_scan_ms += sms;
                graph_walk_ms += ms;
            }
            graph_walks += U;
        }
        done = hc->done;
        if (!done && abort_ms > 0.0 &&
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_call)
                    .count() > abort_ms)
            return fail(PK_ERR_NOT_CONVERGED, "abandoned after %.0f ms (autotuner)", abort_ms);
    }
    if (d.total > 0 && hc->done == 1 && hc->passes_done >= 1) {
        g_last_passes.valid = true;
        g_last_passes.key = key0;
        g_last_passes.passes = hc->passes_done;
    }
    if (d.total > 0)
        HIP_TRY(unpermute_results(P, L, actions, shipped, setup_scr,
                                  unpermute_fits(d.max_T, d.N - 1), st));
    HIP_TRY(hipMemcpyAsync(hc, L.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    // last changed pass per trajectory (read straight into stats->passes without a host
    // buffer of our own when nothing may be allocated)
    std::vector<int32_t> lcp;
    int32_t *lcp_host = stats ? stats->passes : nullptr;
    if (!noalloc) {
        lcp.resize(d.n_traj);
        lcp_host = lcp.data();
    }
    if (lcp_host)
        HIP_TRY(hipMemcpyAsync(lcp_host, L.traj_lcp, d.n_traj * sizeof(int32_t),
                               hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (stats) {
        if (stats->passes)
            for (int b = 0; b < d.n_traj; ++b) stats->passes[b] = lcp_host[b] + 1;
        stats->passes_max = d.total > 0 ? hc->passes_done : 1;
        stats->block_len = o.partition ? 0 : B;
        stats->walk_waves = policy->kind == PK_POLICY_MLP ? waves : 0;
        unsigned long long sum[ST_N] = {};
        for (int i = 0; i < STAT_SLOTS; ++i)
            for (int k = 0; k < ST_N; ++k) sum[k] += hc->stat[i][k];
        stats->changed_total = (int64_t)sum[ST_CHANGED];
        stats->runs_walked = (int64_t)sum[ST_RUNS];
        stats->orders_walked = (int64_t)sum[ST_ORDERS];
        stats->near_ties = (int64_t)sum[ST_NEAR_TIES];
        stats->walk_bytes = (int64_t)sum[ST_BYTES];
        stats->walk_flops = (int64_t)sum[ST_FLOPS];
        stats->scan_bytes = (int64_t)sum[ST_SCAN_BYTES];
        stats->walk_ms = graph_walk_ms;
        stats->scan_ms = graph_scan_ms;
        stats->walk_launches = (int64_t)(evs.size() / 3) + graph_walks;
        stats->scan_launches = stats->walk_launches;
        for (size_t i = 0; i + 2 < evs.size(); i += 3) {
            float ms = 0.f, sms = 0.f;
            if (hipEventElapsedTime(&sms, evs[i], evs[i + 1]) == hipSuccess) stats->scan_ms += sms;
            if (hipEventElapsedTime(&ms, evs[i + 1], evs[i + 2]) == hipSuccess) stats->walk_ms += ms;
        }
    }
    for (hipEvent_t e : evs) (void)hipEventDestroy(e);
    if (hc->error & ERR_NO_PROGRESS)
        return fail(PK_ERR_INTERNAL, "walk made no progress (device state inconsistent)");
    if (hc->error) return fail(PK_ERR_INVALID_ARG, "input value out of range (code %d)", hc->error);
    if (d.total > 0 && hc->done != 1)
        return fail(PK_ERR_NOT_CONVERGED, "not converged after %d passes", hc->passes_done);
    return PK_OK;
}

// ---------------------------------------------------------------- block-length autotuner
struct Tuned {
    int block_len = 0;
    int waves = 4; // learned walk: waves per workgroup
};
std::mutex g_tune_mu;
std::map<std::string, Tuned> g_tune;
bool g_tune_loaded = false;

std::string tune_key(const Dims &d, const pk_policy *po)
{
    int tb = 0;
    while ((1ll << tb) < std::max<int64_t>(d.total, 1)) ++tb;
    int mb = 0;
    while ((1ll << mb) < std::max<int64_t>(d.max_T, 1)) ++mb;
    char buf[160];
    snprintf(buf, sizeof buf, "%s/N%d/R%d/K%d/total2^%d/maxT2^%d",
             po->kind == PK_POLICY_MLP ? "mlp" : "greedy", d.N, d.R, d.K, tb, mb);
    return buf;
}

// The results file beside the library: what the autotuner recorded on MI355X.
std::string shipped_tune_path()
{
    Dl_info info;
    if (!dladdr((void *)&shipped_tune_path, &info) || !info.dli_fname) return "";
    std::string p = info.dli_fname;
    const size_t slash = p.rfind('/');
    return (slash == std::string::npos ? std::string(".") : p.substr(0, slash)) +
           "/autotune_mi355x.json";
}

// A flat JSON object {"key": {"block_len": B, "waves": W}, ...} (a bare number is a block
// length).  Entries already held are kept.
void tune_read_locked(const std::string &path)
{
    FILE *f = fopen(path.c_str(), "r");
    if (!f) return;
    std::string txt;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, n);
    fclose(f);
    size_t i = txt.find('{');
    while (i != std::string::npos && (i = txt.find('"', i + 1)) != std::string::npos) {
        const size_t j = txt.find('"', i + 1);
        if (j == std::string::npos) break;
        const std::string key = txt.substr(i + 1, j - i - 1);
        size_t c = txt.find(':', j);
        if (c == std::string::npos) break;
        ++c;
        while (c < txt.size() && isspace((unsigned char)txt[c])) ++c;
        Tuned t;
        if (c < txt.size() && txt[c] == '{') {
            const size_t e = txt.find('}', c);
            if (e == std::string::npos) break;
            const std::string obj = txt.substr(c, e - c);
            const size_t pb = obj.find("\"block_len\"");
            const size_t pw = obj.find("\"waves\"");
            if (pb != std::string::npos) t.block_len = atoi(obj.c_str() + obj.find(':', pb) + 1);
            if (pw != std::string::npos) t.waves = atoi(obj.c_str() + obj.find(':', pw) + 1);
            i = e;
        } else {
            t.block_len = atoi(txt.c_str() + c);
            i = c;
        }
        if (t.block_len > 0 && (t.waves == 4 || t.waves == 8) && !g_tune.count(key))
            g_tune[key] = t;
    }
}

void tune_load_locked()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = getenv("PICARD_AUTOTUNE_CACHE");
    if (path) tune_read_locked(path);
    else tune_read_locked(shipped_tune_path());
}

void tune_save_locked()
{
    const char *path = getenv("PICARD_AUTOTUNE_CACHE");
    if (!path) return;
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;
    fputs("{", f);
    bool firstk = true;
    for (auto &kv : g_tune) {
        fprintf(f, "%s\n  \"%s\": {\"block_len\": %d, \"waves\": %d}", firstk ? "" : ",",
                kv.first.c_str(), kv.second.block_len, kv.second.waves);
        firstk = false;
    }
    fputs("\n}\n", f);
    fclose(f);
    rename(tmp.c_str(), path);
}

// The cached choice for this problem, if any.
bool tune_lookup(const Dims &d, const pk_policy *po, Tuned *t)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_tune.find(tune_key(d, po));
    if (it == g_tune.end()) return false;
    *t = it->second;
    return true;
}

// Times candidates on this instance and keeps the fastest.  Outputs of the trial runs go
// to `actions`, which the caller overwrites.
//  Greedy: every block length of the ladder, best of three rounds after a warm-up.
//  MLP (whole simulations take seconds at scale): from 2048 upwards while the time falls,
//  then downwards if 2048 stayed best; a candidate is abandoned as soon as it has taken
//  longer than the best so far; then 8 waves per workgroup at the best length.  Short
//  problems (under 0.2 s a run) keep the better of two runs per candidate.
pk_status autotune_block(const pk_problem *problem, const Dims &d, const pk_policy *po,
                         void *ws, size_t ws_bytes, int32_t *actions, hipStream_t st,
                         Tuned *best)
{
    const std::string key = tune_key(d, po);
    if (tune_lookup(d, po, best)) return PK_OK;
    pk_picard_opts o = {};
    o.use_frontier = 1;
    auto run_ms = [&](int B, int waves, double abort_ms, double *ms) -> pk_status {
        o.walk_waves = waves;
        o.graph_unroll = po->kind == PK_POLICY_MLP ? 2 : 0;
        HIP_TRY(hipStreamSynchronize(st));
        const auto t0 = std::chrono::steady_clock::now();
        pk_status s = picard_run(problem, d, po, o, B, ws, ws_bytes, actions, nullptr, nullptr,
                                 nullptr, st, false, abort_ms);
        HIP_TRY(hipStreamSynchronize(st));
        *ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                  .count();
        if (s == PK_ERR_NOT_CONVERGED && abort_ms > 0.0) {
            g_err[0] = 0;
            *ms = 1e30; // abandoned
            return PK_OK;
        }
        return s;
    };
    Tuned pick;
    if (po->kind == PK_POLICY_MLP) {
        static const int ladder[] = {256, 512, 1024, 2048, 4096, 8192, 16384, 32768};
        constexpr int NL = (int)(sizeof(ladder) / sizeof(ladder[0]));
        auto usable = [&](int i) {
            return i >= 0 && i < NL && (ladder[i] <= 2 * std::max<int64_t>(d.total, 1) || i == 0) &&
                   ws_bytes >= picard_bytes(d, po, ladder[i]);
        };
        int i0 = 3; // 2048
        while (i0 > 0 && !usable(i0)) --i0;
        double t = 0.0, tb = 0.0;
        pk_status s = run_ms(ladder[i0], 4, 0.0, &t); // also the warm-up
        if (s != PK_OK) return s;
        const bool twice = t < 200.0;
        auto measure = [&](int B, int waves, double abort, double *out) -> pk_status {
            pk_status r = run_ms(B, waves, abort, out);
            if (r != PK_OK || !twice) return r;
            double again = 0.0;
            r = run_ms(B, waves, abort, &again);
            *out = std::min(*out, again);
            return r;
        };
        if ((s = measure(ladder[i0], 4, 0.0, &tb)) != PK_OK) return s;
        int bi = i0;
        for (int i = i0 + 1; usable(i); ++i) { // upwards
            if ((s = measure(ladder[i], 4, tb, &t)) != PK_OK) return s;
            if (t >= tb) break;
            tb = t;
            bi = i;
        }
        if (bi == i0)
            for (int i = i0 - 1; usable(i); --i) { // downwards
                if ((s = measure(ladder[i], 4, tb, &t)) != PK_OK) return s;
                if (t >= tb) break;
                tb = t;
                bi = i;
            }
        pick.block_len = ladder[bi];
        if ((s = measure(pick.block_len, 8, tb, &t)) != PK_OK) return s;
        if (t < tb) pick.waves = 8;
    } else {
        static const int cands[] = {64, 128, 256, 384, 512, 768, 1024, 1536, 2048, 4096, 8192, 16384, 65536};
        constexpr int NC = (int)(sizeof(cands) / sizeof(cands[0]));
        bool usable[NC];
        for (int i = 0; i < NC; ++i)
            usable[i] = (cands[i] <= 2 * std::max<int64_t>(d.total, 1) || i == 0) &&
                        ws_bytes >= picard_bytes(d, po, cands[i]);
        // warm-up (clocks ramp up on an idle GPU), then rounds over all candidates in turn
        // so that drift affects every candidate alike; each keeps its best time
        const int warm_b = ws_bytes >= picard_bytes(d, po, DEFAULT_BLOCK_GREEDY) ? DEFAULT_BLOCK_GREEDY : cands[0];
        double spent = 0.0;
        for (int k = 0; k < 200 && spent < 300.0; ++k) {
            double ms = 0.0;
            pk_status s = run_ms(warm_b, 4, 0.0, &ms);
            if (s != PK_OK) return s;
            spent += ms;
        }
        double t[NC];
        for (int i = 0; i < NC; ++i) t[i] = 1e30;
        for (int round = 0; round < 3; ++round)
            for (int i = 0; i < NC; ++i) {
                if (!usable[i]) continue;
                double ms = 0.0;
                pk_status s = run_ms(cands[i], 4, 0.0, &ms);
                if (s != PK_OK) return s;
                t[i] = std::min(t[i], ms);
            }
        double best_ms = 1e30;
        pick.block_len = DEFAULT_BLOCK_GREEDY;
        for (int i = 0; i < NC; ++i)
            if (usable[i] && t[i] < best_ms) {
                best_ms = t[i];
                pick.block_len = cands[i];
            }
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = pick;
    tune_save_locked();
    *best = pick;
    return PK_OK;
}


// ---------------------------------------------------------------- OWMR inventory control
pk_status check_owmr(const pk_owmr_problem *pr, OwmrDev *P)
{
    if (!pr) return fail(PK_ERR_INVALID_ARG, "problem is NULL");
    if (pr->n_retailers < 1 || pr->n_orders < 0 || pr->n_orders >= (1ll << 31) - 1)
        return fail(PK_ERR_SHAPE, "need N >= 1 and 0 <= T < 2^31 (N=%d T=%lld)", pr->n_retailers,
                    (long long)pr->n_orders);
    if (pr->n_retailers > (1 << 24)) return fail(PK_ERR_SHAPE, "N=%d exceeds 2^24", pr->n_retailers);
    if (pr->S0 < 0 || pr->x0_init < 0 || pr->S0 >= (1ll << 40) || pr->x0_init >= (1ll << 40))
        return fail(PK_ERR_INVALID_ARG, "S0 and x0_init must be in [0, 2^40)");
    if (!pr->s_ret || !pr->S_ret || !pr->cap || !pr->x_init ||
        (pr->n_orders > 0 && (!pr->retailer || !pr->demand)))
        return fail(PK_ERR_INVALID_ARG, "a problem array is NULL");
    P->N = pr->n_retailers;
    P->T = pr->n_orders;
    P->retailer = pr->retailer;
    P->demand = pr->demand;
    P->s_ret = pr->s_ret;
    P->S_ret = pr->S_ret;
    P->cap = pr->cap;
    P->x_init = pr->x_init;
    P->s0 = pr->s0;
    P->S0 = pr->S0;
    P->x0_init = pr->x0_init;
    return PK_OK;
}

struct OwmrWs {
    int32_t *keys, *keys_alt, *vals, *vals_alt, *sd, *cnt, *err, *fx;
    int64_t *V, *S, *rq, *fx0v, *x0, *sink;
    unsigned long long *resets;
    OwmrCtl *ctl;
    void *rtmp, *stmp;
};

size_t carve_owmr(char *base, const OwmrDev &P, OwmrWs *w)
{
    Carver c{base};
    const int64_t T = std::max<int64_t>(P.T, 1);
    w->ctl = c.take<OwmrCtl>(1);
    w->err = c.take<int32_t>(4);
    w->x0 = c.take<int64_t>(1);
    w->resets = c.take<unsigned long long>(1);
    w->keys = c.take<int32_t>(T);
    w->keys_alt = c.take<int32_t>(T);
    w->vals = c.take<int32_t>(T);
    w->vals_alt = c.take<int32_t>(T);
    w->sd = c.take<int32_t>(T);
    w->cnt = c.take<int32_t>((int64_t)P.N + 1);
    w->fx = c.take<int32_t>(P.N);
    w->V = c.take<int64_t>(T);
    w->S = c.take<int64_t>(T);
    w->rq = c.take<int64_t>(T + 1);
    w->fx0v = c.take<int64_t>(P.N);
    w->sink = c.take<int64_t>(64);
    w->rtmp = c.take<char>((int64_t)owmr_radix_tmp(T));
    w->stmp = c.take<char>((int64_t)std::max(scan_tmp_bytes(T), scan_tmp_bytes((int64_t)P.N + 1)));
    return c.off + 256;
}

// ---------------------------------------------------------------- node capacity
static_assert(sizeof(pk_cap_policy) == 32, "pk_cap_policy layout");
constexpr int DEFAULT_BLOCK_CAP = 96; // fastest of 32..255 on the 1e6-order capacity workload

pk_status check_capacity_problem(const pk_problem *pr, const int32_t *capacity, Dims *d)
{
    pk_status s = check_problem(pr, d);
    if (s != PK_OK) return s;
    if (d->n_traj != 1) return fail(PK_ERR_UNSUPPORTED, "capacity runs take one trajectory");
    if (d->N > CAP_NPAD) return fail(PK_ERR_UNSUPPORTED, "capacity runs take N <= %d", CAP_NPAD);
    if (!capacity) return fail(PK_ERR_INVALID_ARG, "capacity is NULL");
    return PK_OK;
}

// The policy of a capacity run into the plan (NULL: greedy).
pk_status set_cap_policy(const pk_cap_policy *p, CapPlan &L)
{
    L.pol = CAP_GREEDY;
    L.gnum = 0;
    L.gden = 1;
    L.glow = 0;
    L.bid_inv = L.bid_cap = nullptr;
    if (!p) return PK_OK;
    if (p->gamma_num < 0 || p->gamma_num > 1000 || p->gamma_den < 1 || p->gamma_den > 1000)
        return fail(PK_ERR_INVALID_ARG, "gamma must be num/den with 0 <= num <= 1000, "
                                        "1 <= den <= 1000 (got %d/%d)", p->gamma_num, p->gamma_den);
    if (p->gamma_low < 0) return fail(PK_ERR_INVALID_ARG, "gamma_low must be >= 0 (got %d)", p->gamma_low);
    if (p->reserved != 0) return fail(PK_ERR_INVALID_ARG, "pk_cap_policy.reserved must be 0");
    const bool bids = p->bid_inv || p->bid_cap;
    if (bids && p->gamma_num != 0)
        return fail(PK_ERR_INVALID_ARG, "bid prices take gamma_num = 0");
    L.gnum = p->gamma_num;
    L.gden = p->gamma_den;
    L.glow = p->gamma_low;
    L.bid_inv = p->bid_inv;
    L.bid_cap = p->bid_cap;
    L.pol = bids ? CAP_BID : p->gamma_num > 0 ? CAP_GAMMA : CAP_GREEDY;
    return PK_OK;
}

struct CapWs {
    CapPlan L;
    int32_t *keys, *vals, *keys_alt, *vals_alt, *first, *used, *state;
    void *tmp;
};

// Carves (or measures, with base == nullptr) a capacity run's workspace.
size_t carve_cap(char *base, const Dims &d, int B, bool picard, CapWs *w)
{
    Carver c{base};
    CapWs x = {};
    const int64_t T = d.total;
    const int64_t nblk = std::max<int64_t>(1, (T + B - 1) / B);
    const int64_t max_pieces = d.K + T / CAP_PIECE + 1;
    x.L.ctl = c.take<CapCtl>(1);
    x.L.keyT = c.take<uint32_t>((int64_t)d.R * CAP_NPAD);
    x.used = c.take<int32_t>(CAP_NPAD);
    if (picard) {
        x.L.perm = c.take<int32_t>(T);
        x.L.seg_off = c.take<int32_t>(d.K + 1);
        x.L.slot = c.take<int32_t>(T);
        x.L.sid = c.take<int32_t>(T);
        x.L.srow = c.take<int32_t>(T);
        x.L.piece_off = c.take<int32_t>(d.K + 1);
        x.L.piece = c.take<int4>(max_pieces);
        x.L.pc = c.take<int32_t>(max_pieces * CAP_NPAD);
        x.L.H = c.take<int32_t>((int64_t)d.N * nblk);
        x.L.capE = c.take<int32_t>(nblk * d.N);
        x.L.X = c.take<uint8_t>(std::max<int64_t>(T, 1) * CAP_NPAD);
        x.L.P = c.take<uint8_t>(T);
        x.L.skuchg = c.take<int32_t>(d.K);
        x.L.chg = c.take<int32_t>(CAP_GROUP);
        x.keys = c.take<int32_t>(T);
        x.vals = c.take<int32_t>(T);
        x.keys_alt = c.take<int32_t>(T);
        x.vals_alt = c.take<int32_t>(T);
        x.first = c.take<int32_t>(T);
        x.tmp = c.take<char>((int64_t)std::max(radix_tmp_bytes(T),
                                               scan_tmp_bytes(std::max<int64_t>(T, d.K + 1))));
    } else {
        x.state = c.take<int32_t>((int64_t)d.K * d.N);
    }
    x.L.T = (int32_t)T;
    x.L.N = d.N;
    x.L.K = d.K;
    x.L.R = d.R;
    x.L.B = B;
    x.L.nblk = (int32_t)nblk;
    x.L.max_pieces = max_pieces;
    if (w) *w = x;
    return c.off + 256;
}

void cap_bind(CapPlan &L, const pk_problem *pr, const int32_t *capacity, int32_t *actions)
{
    L.sku = pr->sku;
    L.region = pr->region;
    L.qty = pr->qty;
    L.x0 = pr->init_inv;
    L.cost = pr->cost;
    L.cap0 = capacity;
    L.alpha = actions;
}

pk_status cap_errors(const CapCtl &h)
{
    if (!h.error) return PK_OK;
    return fail(PK_ERR_INVALID_ARG,
                "invalid input (bits %#x: 1 quantity != 1, 2 SKU, 4 region, 8 negative stock, "
                "16 negative capacity, 32 cost outside [0, 2^24), 64 initial cache outside [-1, N), "
                "128 bid price outside [0, 2^24))",
                h.error);
}

} // namespace

extern "C" {

const char *pk_last_error(void) { return g_err; }

pk_status pk_owmr_workspace_size(const pk_owmr_problem *problem, size_t *bytes)
{
    g_err[0] = 0;
    OwmrDev P;
    pk_status s = check_owmr(problem, &P);
    if (s != PK_OK) return s;
    if (!bytes) return fail(PK_ERR_INVALID_ARG, "bytes is NULL");
    OwmrWs w;
    *bytes = carve_owmr(nullptr, P, &w);
    return PK_OK;
}

pk_status pk_owmr_serial_simulate(const pk_owmr_problem *problem, void *ws, size_t ws_bytes,
                                  int32_t *q, int32_t *reset, int32_t *final_x,
                                  int64_t *final_x0, int64_t *resets, void *stream)
{
    g_err[0] = 0;
    OwmrDev P;
    pk_status s = check_owmr(problem, &P);
    if (s != PK_OK) return s;
    if (P.T > 0 && (!q || !reset)) return fail(PK_ERR_INVALID_ARG, "q/reset is NULL");
    OwmrWs w;
    if (!ws || ws_bytes < carve_owmr(nullptr, P, &w))
        return fail(PK_ERR_WORKSPACE, "workspace too small");
    carve_owmr(align_ws(ws), P, &w);
    hipStream_t st = (hipStream_t)stream;
    int32_t *perm = nullptr;
    HIP_TRY(owmr_launch_setup(P, w.keys, w.keys_alt, w.vals, w.vals_alt, w.rtmp, w.cnt, w.stmp,
                              w.sd, w.err, &perm, st)); // (input checks; the sort is unused)
    int32_t herr = 0;
    HIP_TRY(hipMemcpyAsync(&herr, w.err, sizeof herr, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (herr) return fail(PK_ERR_INVALID_ARG, "an OWMR input is out of range");
    if (P.N > 40 * 1024) return fail(PK_ERR_SHAPE, "the serial sweep keeps N <= 40960 stocks in LDS");
    HIP_TRY(owmr_launch_serial(P, q, reset, w.x0, final_x ? final_x : w.fx, w.resets, st));
    int64_t hx0 = 0;
    unsigned long long hr = 0;
    HIP_TRY(hipMemcpyAsync(&hx0, w.x0, sizeof hx0, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&hr, w.resets, sizeof hr, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (final_x0) *final_x0 = hx0;
    if (resets) *resets = (int64_t)hr;
    return PK_OK;
}

pk_status pk_owmr_picard_simulate(const pk_owmr_problem *problem, int32_t max_passes,
                                  const int32_t *init_q, const int32_t *init_reset, void *ws,
                                  size_t ws_bytes, int32_t *q, int32_t *reset, int32_t *final_x,
                                  int64_t *final_x0, int32_t *passes, int64_t *changed,
                                  int64_t *caches, void *stream)
{
    g_err[0] = 0;
    OwmrDev P;
    pk_status s = check_owmr(problem, &P);
    if (s != PK_OK) return s;
    if (P.T > 0 && (!q || !reset)) return fail(PK_ERR_INVALID_ARG, "q/reset is NULL");
    if (!passes) return fail(PK_ERR_INVALID_ARG, "passes is NULL");
    if (max_passes < 0) return fail(PK_ERR_INVALID_ARG, "max_passes < 0");
    if ((init_q == nullptr) != (init_reset == nullptr))
        return fail(PK_ERR_INVALID_ARG, "give both init_q and init_reset, or neither");
    const int32_t mp = max_passes > 0 ? max_passes : (int32_t)std::min<int64_t>(P.T + 1, 0x7ffffff0);
    if ((changed || caches) && max_passes <= 0)
        return fail(PK_ERR_INVALID_ARG, "recording passes needs max_passes > 0");
    OwmrWs w;
    if (!ws || ws_bytes < carve_owmr(nullptr, P, &w))
        return fail(PK_ERR_WORKSPACE, "workspace too small");
    carve_owmr(align_ws(ws), P, &w);
    hipStream_t st = (hipStream_t)stream;
    int32_t *perm = nullptr;
    HIP_TRY(owmr_launch_setup(P, w.keys, w.keys_alt, w.vals, w.vals_alt, w.rtmp, w.cnt, w.stmp,
                              w.sd, w.err, &perm, st));
    HIP_TRY(owmr_launch_init(P, init_q, init_reset, w.V, w.ctl, mp, st));
    int32_t herr = 0;
    HIP_TRY(hipMemcpyAsync(&herr, w.err, sizeof herr, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (herr) return fail(PK_ERR_INVALID_ARG, "an OWMR input is out of range");
    // passes go out eight at a time (every kernel returns at once after convergence),
    // one at a time when each pass's cache is recorded
    const int U = caches ? 1 : 8;
    OwmrCtl hc = {};
    int launched = 0;
    while (launched < mp) {
        const int u = std::min(U, mp - launched);
        for (int i = 0; i < u; ++i)
            HIP_TRY(owmr_launch_pass(P, w.ctl, perm, w.sd, w.cnt, w.V, w.S, w.rq, w.stmp, w.fx0v,
                                     final_x ? final_x : w.fx,
                                     caches ? caches + (int64_t)(launched + i) * P.T : nullptr,
                                     w.sink, st));
        launched += u;
        HIP_TRY(hipMemcpyAsync(&hc, w.ctl, sizeof hc, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (changed)
            for (int k = launched - u; k < launched && k < (hc.done ? hc.passes_done : launched); ++k)
                changed[k] = (int64_t)hc.changed_log[k & 7];
        if (hc.done) break;
    }
    *passes = hc.done ? hc.passes_done : launched;
    if (P.T > 0) HIP_TRY(owmr_launch_unpack(P, w.V, q, reset, st));
    if (final_x0) {
        int64_t x0 = P.x0_init;
        if (P.T > 0) { // the last order's retailer sees the exact central stock after it
            int32_t nl = 0;
            HIP_TRY(hipMemcpyAsync(&nl, P.retailer + P.T - 1, sizeof nl, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            HIP_TRY(hipMemcpyAsync(&x0, w.fx0v + nl, sizeof x0, hipMemcpyDeviceToHost, st));
        }
        HIP_TRY(hipStreamSynchronize(st));
        *final_x0 = x0;
    }
    HIP_TRY(hipStreamSynchronize(st));
    if (hc.done != 1) return fail(PK_ERR_NOT_CONVERGED, "not converged after %d passes", *passes);
    return PK_OK;
}

const char *pk_version(void) { return "libpicard 0.1 (gfx950)"; }

pk_status pk_workspace_size(const pk_problem *problem, const pk_policy *policy,
                            const pk_picard_opts *opts, size_t *bytes)
{
    Dims d;
    pk_status s = check_problem(problem, &d);
    if (s != PK_OK) return s;
    if ((s = check_policy(policy)) != PK_OK) return s;
    if (!bytes) return fail(PK_ERR_INVALID_ARG, "bytes is NULL");
    int B = opts && opts->block_len > 0 ? opts->block_len : MIN_AUTOTUNE_BLOCK;
    if (policy->kind == PK_POLICY_MLP && !(opts && opts->block_len > 0)) B = MIN_AUTOTUNE_BLOCK;
    if (opts && opts->partition) B = 1;
    *bytes = std::max(picard_bytes(d, policy, B), serial_bytes(d)) +
             (((size_t)std::max<int64_t>(d.total, 1) * 4 + 255) & ~(size_t)255) + 512;
    if (policy->kind == PK_POLICY_MLP) *bytes = std::max(*bytes, grad_bytes(d, policy));
    return PK_OK;
}

pk_status pk_serial_simulate(const pk_problem *problem, const pk_policy *policy, void *ws,
                             size_t ws_bytes, int32_t *actions, int32_t *shipped,
                             int32_t *final_inv, int32_t validate, void *stream)
{
    g_err[0] = 0;
    Dims d;
    pk_status s = check_problem(problem, &d);
    if (s != PK_OK) return s;
    if ((s = check_policy(policy)) != PK_OK) return s;
    if (d.total > 0 && !actions) return fail(PK_ERR_INVALID_ARG, "actions is NULL");
    if (!ws || ws_bytes < serial_bytes(d)) return fail(PK_ERR_WORKSPACE, "workspace too small");
    hipStream_t st = (hipStream_t)stream;
    Carver c{align_ws(ws)};
    int64_t *to = c.take<int64_t>(d.n_traj + 1);
    void *pos = c.take<char>(
        (int64_t)std::max(pos_bytes(d.N, d.R, d.n_traj), costT_bytes(d.N, d.R, d.n_traj)));
    int32_t *state = final_inv ? final_inv : c.take<int32_t>((int64_t)d.n_traj * d.K * d.N);
    HIP_TRY(hipMemcpyAsync(to, problem->traj_offsets, (d.n_traj + 1) * sizeof(int64_t),
                           hipMemcpyHostToDevice, st));
    Prob P = make_prob(problem, d, to);
    HIP_TRY(hipMemcpyAsync(state, problem->init_inv, (size_t)d.n_traj * d.K * d.N * 4,
                           hipMemcpyDeviceToDevice, st));
    (void)validate;
    if (policy->kind == PK_POLICY_MLP) {
        HIP_TRY(setup_costT(P, policy->params, (float *)pos, st));
        HIP_TRY(launch_serial_mlp(P, policy->params, policy->n_hidden_layers, (const float *)pos,
                                  state, actions, shipped, st));
    } else {
        HIP_TRY(setup_pos(P, pos, nullptr, st));
        HIP_TRY(launch_serial_greedy(P, pos, state, actions, shipped, st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    return PK_OK;
}

pk_status pk_picard_simulate(const pk_problem *problem, const pk_policy *policy,
                             const pk_picard_opts *opts, void *ws, size_t ws_bytes,
                             int32_t *actions, int32_t *shipped, int32_t *final_inv,
                             pk_stats *stats, void *stream)
{
    g_err[0] = 0;
    Dims d;
    pk_status s = check_problem(problem, &d);
    if (s != PK_OK) return s;
    if ((s = check_policy(policy)) != PK_OK) return s;
    if (d.total > 0 && !actions) return fail(PK_ERR_INVALID_ARG, "actions is NULL");
    pk_picard_opts o = {};
    o.use_frontier = 1;
    if (opts) o = *opts;
    if (o.block_len < 0 || o.max_passes < 0 || o.graph_unroll < 0)
        return fail(PK_ERR_INVALID_ARG, "negative option");
    if (o.walk_waves != 0 && o.walk_waves != 4 && o.walk_waves != 8)
        return fail(PK_ERR_INVALID_ARG, "walk_waves must be 0, 4 or 8 (got %d)", o.walk_waves);
    if (o.partition) o.block_len = 1; // sizes the plan for one run per order, the most
                                      // a partition makes
    int B = o.block_len;
    Tuned t;
    const bool tuned = tune_lookup(d, policy, &t);
    if (B == 0 && policy->kind == PK_POLICY_MLP) // learned: the recorded choice, else the
        B = tuned ? t.block_len : DEFAULT_BLOCK_MLP; // default (tuning takes minutes)
    if (B == 0) {
        s = autotune_block(problem, d, policy, ws, ws_bytes, actions, (hipStream_t)stream, &t);
        if (s != PK_OK) return s;
        B = t.block_len;
    }
    if (o.walk_waves == 0) o.walk_waves = tuned && t.block_len == B ? t.waves : 4;
    return picard_run(problem, d, policy, o, B, ws, ws_bytes, actions, shipped, final_inv, stats,
                      (hipStream_t)stream);
}

pk_status pk_picard_simulate_noalloc(const pk_problem *problem, const pk_policy *policy,
                                     const pk_picard_opts *opts, int32_t *actions,
                                     int32_t *shipped, int32_t *final_inv, pk_stats *stats,
                                     void *stream)
{
    g_err[0] = 0;
    Dims d;
    pk_status s = check_problem(problem, &d);
    if (s != PK_OK) return s;
    if ((s = check_policy(policy)) != PK_OK) return s;
    if (d.total > 0 && !actions) return fail(PK_ERR_INVALID_ARG, "actions is NULL");
    pk_picard_opts o = {};
    o.use_frontier = 1;
    if (opts) o = *opts;
    if (o.block_len < 0 || o.max_passes < 0 || o.graph_unroll < 0)
        return fail(PK_ERR_INVALID_ARG, "negative option");
    if (o.walk_waves != 0 && o.walk_waves != 4 && o.walk_waves != 8)
        return fail(PK_ERR_INVALID_ARG, "walk_waves must be 0, 4 or 8 (got %d)", o.walk_waves);
    if (stats && stats->timing)
        return fail(PK_ERR_UNSUPPORTED, "timing needs HIP events, which this entry point "
                                        "does not create");
    if (o.partition) o.block_len = 1;
    int B = o.block_len;
    if (B == 0) B = policy->kind == PK_POLICY_MLP ? DEFAULT_BLOCK_MLP : DEFAULT_BLOCK_GREEDY;
    const size_t need = picard_bytes(d, policy, B);
    if (need > (size_t)PK_NOALLOC_SCRATCH_BYTES)
        return fail(PK_ERR_WORKSPACE,
                    "this problem needs %zu bytes of scratch, more than the %zu bytes of the "
                    "static buffer (use pk_picard_simulate with a workspace)",
                    need, (size_t)PK_NOALLOC_SCRATCH_BYTES);
    void *ptr = nullptr;
    if ((s = scratch_on_current_device(&ptr)) != PK_OK) return s;
    return picard_run(problem, d, policy, o, B, ptr, PK_NOALLOC_SCRATCH_BYTES, actions, shipped,
                      final_inv, stats, (hipStream_t)stream, /*noalloc=*/true);
}

pk_status pk_policy_grad(const pk_problem *problem, const pk_policy *policy,
                         const int32_t *actions, const float *advantages, float *logp,
                         float *grad, double *objective, void *ws, size_t ws_bytes,
                         int32_t validate, void *stream)
{
    g_err[0] = 0;
    Dims d;
    pk_status s = check_problem(problem, &d);
    if (s != PK_OK) return s;
    if ((s = check_policy(policy)) != PK_OK) return s;
    if (policy->kind != PK_POLICY_MLP) return fail(PK_ERR_INVALID_ARG, "policy_grad needs the MLP policy");
    if (d.total > 0 && (!actions || !advantages))
        return fail(PK_ERR_INVALID_ARG, "actions/advantages is NULL");
    if (!ws || ws_bytes < grad_bytes(d, policy))
        return fail(PK_ERR_WORKSPACE, "workspace too small: need %zu bytes, got %zu",
                    grad_bytes(d, policy), ws_bytes);
    hipStream_t st = (hipStream_t)stream;
    Carver c{align_ws(ws)};
    Plan L;
    int64_t *to;
    void *setup_scr;
    carve_plan(c, d, policy, GRAD_BLOCK, &L, &to, &setup_scr);
    float *logp_sorted = c.take<float>(d.total);
    double *part = c.take<double>((int64_t)grad_part_bytes(GRAD_MAX_WG, d.R, policy->n_hidden_layers) / 8);
    double *obj_dev = c.take<double>(1);
    const Sizes sz = plan_sizes(d, GRAD_BLOCK);
    HIP_TRY(hipMemcpyAsync(to, problem->traj_offsets, (d.n_traj + 1) * sizeof(int64_t),
                           hipMemcpyHostToDevice, st));
    Prob P = make_prob(problem, d, to);
    HIP_TRY(setup_ctl(L, d.n_traj, 1, st));
    // two workgroups per CU where their LDS fits (two waves per SIMD), else one
    const int n_wg = std::min(GRAD_MAX_WG, std::max(1, num_cus() * grad_wg_per_cu(d.N)));
    if (d.total > 0) {
        // states of the fixed actions: the actions are the cache, its consumption scanned
        HIP_TRY(setup_plan(P, L, actions, validate, true, (int32_t)sz.n_seg_max, setup_scr, st));
        HIP_TRY(setup_costT(P, policy->params, L.costT, st));
        HIP_TRY(launch_consume(P, L, sz.n_split_max, st));
        HIP_TRY(launch_scan_entry(P, L, (int)sz.n_seg_max, false, st));
        HIP_TRY(launch_grad(P, L, policy->params, policy->n_hidden_layers, L.costT, advantages,
                            logp_sorted, part, n_wg, grad, obj_dev, logp, st));
    } else {
        HIP_TRY(hipMemsetAsync(obj_dev, 0, sizeof(double), st));
        if (grad)
            HIP_TRY(hipMemsetAsync(grad, 0,
                                   ((size_t)d.R * 16 + 64 * 18 + 64 + 64 + 1 +
                                    (policy->n_hidden_layers == 2 ? 64 * 64 + 64 : 0)) * 4, st));
    }
    Ctl *hc = g_pinned.get();
    if (!hc) return fail(PK_ERR_HIP, "pinned host allocation failed");
    double objv = 0.0;
    HIP_TRY(hipMemcpyAsync(hc, L.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&objv, obj_dev, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (objective) *objective = objv;
    if (d.total > 0 && hc->error)
        return fail(PK_ERR_INVALID_ARG, "input or action out of range / infeasible (code %d)",
                    hc->error);
    return PK_OK;
}

pk_status pk_policy_scores(const pk_problem *problem, const pk_policy *policy, int32_t traj,
                           int32_t region, const int32_t *inv_row, float *scores, void *ws,
                           size_t ws_bytes, void *stream)
{
    g_err[0] = 0;
    Dims d;
    pk_status s = check_problem(problem, &d);
    if (s != PK_OK) return s;
    if ((s = check_policy(policy)) != PK_OK) return s;
    if (policy->kind != PK_POLICY_MLP) return fail(PK_ERR_INVALID_ARG, "scores need the MLP policy");
    if (traj < 0 || traj >= d.n_traj || region < 0 || region >= d.R)
        return fail(PK_ERR_INVALID_ARG, "traj or region out of range");
    if (!inv_row || !scores) return fail(PK_ERR_INVALID_ARG, "inv_row/scores is NULL");
    const size_t need = costT_bytes(d.N, d.R, d.n_traj) + 1024;
    if (!ws || ws_bytes < need) return fail(PK_ERR_WORKSPACE, "workspace too small");
    hipStream_t st = (hipStream_t)stream;
    Carver c{align_ws(ws)};
    float *costT = c.take<float>((int64_t)costT_bytes(d.N, d.R, d.n_traj) / 4);
    Prob P = make_prob(problem, d, nullptr);
    HIP_TRY(setup_costT(P, policy->params, costT, st));
    HIP_TRY(launch_scores(P, policy->params, policy->n_hidden_layers, costT, traj, region, inv_row,
                          scores, st));
    HIP_TRY(hipStreamSynchronize(st));
    return PK_OK;
}

pk_status pk_autotune(const pk_problem *problem, const pk_policy *policy, void *ws,
                      size_t ws_bytes, int32_t *best_block_len, void *stream)
{
    g_err[0] = 0;
    Dims d;
    pk_status s = check_problem(problem, &d);
    if (s != PK_OK) return s;
    if ((s = check_policy(policy)) != PK_OK) return s;
    if (!best_block_len) return fail(PK_ERR_INVALID_ARG, "best_block_len is NULL");
    const size_t act_bytes = ((size_t)std::max<int64_t>(d.total, 1) * 4 + 255) & ~(size_t)255;
    if (!ws || ws_bytes < act_bytes + 512) return fail(PK_ERR_WORKSPACE, "workspace too small");
    // trial actions live at the end of the workspace
    char *tail = (char *)ws + ((ws_bytes - act_bytes) & ~(size_t)255);
    Tuned t;
    s = autotune_block(problem, d, policy, ws, (size_t)(tail - (char *)ws), (int32_t *)tail,
                       (hipStream_t)stream, &t);
    if (s != PK_OK) return s;
    *best_block_len = t.block_len;
    return PK_OK;
}

pk_status pk_advantages_workspace_size(const pk_problem *problem, size_t *bytes)
{
    g_err[0] = 0;
    Dims d;
    pk_status s = check_problem(problem, &d);
    if (s != PK_OK) return s;
    if (!bytes) return fail(PK_ERR_INVALID_ARG, "bytes is NULL");
    *bytes = advantages_ws_bytes(d.total, d.n_traj);
    return PK_OK;
}

pk_status pk_reinforce_advantages(const pk_problem *problem, const int32_t *actions,
                                  const int32_t *shipped, int32_t revenue, float *advantages,
                                  int64_t *returns, void *ws, size_t ws_bytes, void *stream)
{
    g_err[0] = 0;
    Dims d;
    pk_status s = check_problem(problem, &d);
    if (s != PK_OK) return s;
    if (d.total > 0 && (!actions || !shipped || !advantages))
        return fail(PK_ERR_INVALID_ARG, "actions/shipped/advantages is NULL");
    const size_t need = advantages_ws_bytes(d.total, d.n_traj);
    if (!ws || ws_bytes < need)
        return fail(PK_ERR_WORKSPACE, "workspace too small: need %zu bytes, got %zu", need,
                    ws_bytes);
    hipStream_t st = (hipStream_t)stream;
    if (returns) HIP_TRY(hipMemsetAsync(returns, 0, (size_t)d.n_traj * sizeof(int64_t), st));
    if (d.total == 0) {
        HIP_TRY(hipStreamSynchronize(st));
        return PK_OK;
    }
    // |r| <= rlim keeps every int64 sum exact: the weighted sum of a trajectory is at most
    // rlim * T (T + 1) / 2 <= 2^62 and the batch prefix at most total * 2^31 < 2^62
    const int64_t T = d.max_T;
    const int64_t tri = T * (T + 1) / 2; // T < 2^31, so no overflow
    const int64_t rlim = std::min<int64_t>(1ll << 31, (1ll << 62) / tri);
    Carver c{align_ws(ws)};
    int64_t *offs = c.take<int64_t>(d.n_traj + 1);
    int64_t *rew = c.take<int64_t>(d.total);
    unsigned long long *wsum = c.take<unsigned long long>(d.n_traj);
    int32_t *err = c.take<int32_t>(1);
    void *tmp = c.take<char>((int64_t)scan_tmp_bytes(d.total));
    HIP_TRY(hipMemcpyAsync(offs, problem->traj_offsets, (d.n_traj + 1) * sizeof(int64_t),
                           hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemsetAsync(wsum, 0, (size_t)d.n_traj * 8, st));
    HIP_TRY(hipMemsetAsync(err, 0, 4, st));
    HIP_TRY(launch_advantages(offs, d.n_traj, d.N, d.R, d.total, problem->region, actions,
                              shipped, problem->cost, revenue, rlim, rew, wsum, err, tmp,
                              advantages, returns, st));
    int32_t herr = 0;
    HIP_TRY(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (herr & 1) return fail(PK_ERR_INVALID_ARG, "an action, region or shipped count is out of range");
    if (herr & 2)
        return fail(PK_ERR_INVALID_ARG, "a reward exceeds %lld in magnitude (int64 sums would overflow)",
                    (long long)rlim);
    return PK_OK;
}

pk_status pk_adam_step(float *params, const float *grad, float *m, float *v, int64_t n,
                       int32_t step, double lr, double beta1, double beta2, double eps,
                       int32_t ascend, void *stream)
{
    g_err[0] = 0;
    if (n < 0) return fail(PK_ERR_INVALID_ARG, "n must be >= 0");
    if (n > 0 && (!params || !grad || !m || !v))
        return fail(PK_ERR_INVALID_ARG, "params/grad/m/v is NULL");
    if (step < 1) return fail(PK_ERR_INVALID_ARG, "step must be >= 1");
    if (!(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0))
        return fail(PK_ERR_INVALID_ARG, "beta1/beta2 must lie in [0, 1)");
    if (!(lr >= 0.0) || !(eps > 0.0)) return fail(PK_ERR_INVALID_ARG, "need lr >= 0 and eps > 0");
    AdamCoef c;
    c.lr = (float)lr;
    c.b1 = (float)beta1;
    c.b2 = (float)beta2;
    c.omb1 = (float)(1.0 - beta1);
    c.omb2 = (float)(1.0 - beta2);
    c.bc1 = (float)(1.0 - std::pow(beta1, (double)step));
    c.bc2 = (float)(1.0 - std::pow(beta2, (double)step));
    c.eps = (float)eps;
    c.dir = ascend ? 1.0f : -1.0f;
    HIP_TRY(launch_adam(params, grad, m, v, n, c, (hipStream_t)stream));
    return PK_OK;
}

pk_status pk_capacity_workspace_size(const pk_problem *problem, const int32_t *capacity,
                                     int32_t block_len, size_t *bytes)
{
    g_err[0] = 0;
    Dims d;
    pk_status s = check_capacity_problem(problem, capacity, &d);
    if (s != PK_OK) return s;
    if (!bytes) return fail(PK_ERR_INVALID_ARG, "bytes is NULL");
    if (block_len < 0 || block_len > CAP_MAX_B)
        return fail(PK_ERR_INVALID_ARG, "block_len must lie in [0, %d]", CAP_MAX_B);
    const int B = block_len ? block_len : DEFAULT_BLOCK_CAP;
    *bytes = std::max(carve_cap(nullptr, d, B, true, nullptr),
                      carve_cap(nullptr, d, B, false, nullptr)) + 256;
    return PK_OK;
}

pk_status pk_serial_simulate_capacity(const pk_problem *problem, const int32_t *capacity,
                                      const pk_cap_policy *policy, void *ws,
                                      size_t ws_bytes, int32_t *actions, int32_t *final_inv,
                                      int32_t *final_cap, void *stream)
{
    g_err[0] = 0;
    Dims d;
    pk_status s = check_capacity_problem(problem, capacity, &d);
    if (s != PK_OK) return s;
    CapPlan pol = {};
    if ((s = set_cap_policy(policy, pol)) != PK_OK) return s;
    if (d.total > 0 && !actions) return fail(PK_ERR_INVALID_ARG, "actions is NULL");
    if (!ws || ws_bytes < carve_cap(nullptr, d, DEFAULT_BLOCK_CAP, false, nullptr))
        return fail(PK_ERR_WORKSPACE, "workspace too small");
    hipStream_t st = (hipStream_t)stream;
    CapWs w;
    carve_cap(align_ws(ws), d, DEFAULT_BLOCK_CAP, false, &w);
    cap_bind(w.L, problem, capacity, actions);
    set_cap_policy(policy, w.L);
    int32_t *state = final_inv ? final_inv : w.state;
    HIP_TRY(cap_check(w.L, nullptr, st));
    CapCtl h;
    HIP_TRY(hipMemcpyAsync(&h, w.L.ctl, sizeof h, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if ((s = cap_errors(h)) != PK_OK) return s;
    HIP_TRY(cap_serial_setup(w.L, st));
    HIP_TRY(hipMemcpyAsync(state, problem->init_inv, (size_t)d.K * d.N * 4,
                           hipMemcpyDeviceToDevice, st));
    HIP_TRY(cap_serial(w.L, state, actions, st));
    if (final_cap) HIP_TRY(cap_finish(w.L, nullptr, final_cap, w.used, st));
    HIP_TRY(hipStreamSynchronize(st));
    return PK_OK;
}

pk_status pk_picard_simulate_capacity(const pk_problem *problem, const int32_t *capacity,
                                      const pk_cap_policy *policy, int32_t block_len, int32_t max_passes,
                                      const int32_t *init_cache, void *ws, size_t ws_bytes,
                                      int32_t *actions, int32_t *final_inv, int32_t *final_cap,
                                      int32_t *passes, int64_t *changed, int32_t *caches,
                                      void *stream)
{
    g_err[0] = 0;
    Dims d;
    pk_status s = check_capacity_problem(problem, capacity, &d);
    if (s != PK_OK) return s;
    if (d.total > 0 && !actions) return fail(PK_ERR_INVALID_ARG, "actions is NULL");
    CapPlan pol = {};
    if ((s = set_cap_policy(policy, pol)) != PK_OK) return s;
    if (block_len < 0 || block_len > CAP_MAX_B)
        return fail(PK_ERR_INVALID_ARG, "block_len must lie in [0, %d]", CAP_MAX_B);
    if (max_passes < 0) return fail(PK_ERR_INVALID_ARG, "max_passes must be >= 0");
    const int B = block_len ? block_len : DEFAULT_BLOCK_CAP;
    const int64_t T = d.total;
    const int32_t mp = max_passes ? max_passes : (int32_t)std::min<int64_t>(T + 1, INT32_MAX);
    if (!ws || ws_bytes < carve_cap(nullptr, d, B, true, nullptr))
        return fail(PK_ERR_WORKSPACE, "workspace too small");
    hipStream_t st = (hipStream_t)stream;
    CapWs w;
    carve_cap(align_ws(ws), d, B, true, &w);
    cap_bind(w.L, problem, capacity, actions);
    set_cap_policy(policy, w.L);
    HIP_TRY(cap_check(w.L, init_cache, st));
    CapCtl h;
    HIP_TRY(hipMemcpyAsync(&h, w.L.ctl, sizeof h, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if ((s = cap_errors(h)) != PK_OK) return s;
    w.L.first = w.first;
    HIP_TRY(cap_setup(w.L, w.keys, w.vals, w.keys_alt, w.vals_alt, w.first, w.tmp, st));
    HIP_TRY(hipMemcpyAsync(&h, w.L.ctl, sizeof h, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    w.L.dmax = std::max(h.max_distinct, 1);
    if (T > 0) {
        if (init_cache)
            HIP_TRY(hipMemcpyAsync(actions, init_cache, (size_t)T * 4, hipMemcpyDeviceToDevice, st));
        else
            HIP_TRY(hipMemsetAsync(actions, 0xff, (size_t)T * 4, st)); // all lost sales (-1)
    }
    // passes go out CAP_GROUP at a time; the host then reads their change counts. A pass
    // after the first one without change is a no-op (nothing lies past its restart point
    // and no SKU changed), so the passes run past convergence leave the result as it is.
    int32_t done_at = 0;
    int32_t cg[CAP_GROUP];
    for (int32_t k0 = 1; k0 <= mp && !done_at; k0 += CAP_GROUP) {
        const int32_t kn = std::min<int32_t>(CAP_GROUP, mp - k0 + 1);
        for (int32_t j = 0; j < kn; ++j) {
            const int32_t k = k0 + j;
            HIP_TRY(cap_pass(w.L, k == 1, st));
            if (caches && T > 0)
                HIP_TRY(hipMemcpyAsync(caches + (int64_t)(k - 1) * T, actions, (size_t)T * 4,
                                       hipMemcpyDeviceToDevice, st));
        }
        HIP_TRY(hipMemcpyAsync(cg, w.L.chg, sizeof cg, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        for (int32_t j = 0; j < kn && !done_at; ++j) {
            const int32_t k = k0 + j;
            const int32_t c = cg[(k - 1) % CAP_GROUP];
            if (changed) changed[k - 1] = c;
            if (c == 0) done_at = k;
        }
    }
    const bool converged = done_at > 0;
    if (passes) *passes = converged ? done_at : mp;
    if (!converged) return fail(PK_ERR_NOT_CONVERGED, "no fixed point after %d passes", mp);
    HIP_TRY(cap_finish(w.L, final_inv, final_cap, w.used, st));
    HIP_TRY(hipStreamSynchronize(st));
    return PK_OK;
}

} // extern "C"

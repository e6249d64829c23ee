// C-ABI entry points of libpicard (declared in include/picard.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "pk_internal.h"

namespace pk {
// setup.hip
hipError_t setup_ctl(Plan &L, int n_traj, int max_passes, hipStream_t st);
hipError_t setup_plan(const Prob &P, Plan &L, const int32_t *init_cache, int validate,
                      bool want_t, int32_t n_seg_max, void *scratch, hipStream_t st);
size_t setup_scratch_bytes(int64_t n);
hipError_t setup_rank(const Prob &P, int16_t *rank, hipStream_t st);
// pass.hip
hipError_t launch_scan_entry(const Prob &P, const Plan &L, int n_seg_max, bool skip_first,
                             hipStream_t st);
hipError_t launch_pass_end(const Plan &L, hipStream_t st);
hipError_t launch_consume(const Prob &P, const Plan &L, int64_t n_split_max, hipStream_t st);
hipError_t launch_unpermute(const Prob &P, const Plan &L, int32_t *actions, int32_t *shipped,
                            hipStream_t st);
// greedy.hip
size_t walk_greedy_lds(int N, int R);
hipError_t launch_walk_greedy(const Prob &P, const Plan &L, int32_t *final_inv, bool has_init,
                              int grid, hipStream_t st);
hipError_t launch_serial_greedy(const Prob &P, const int16_t *rank, int32_t *state,
                                int32_t *actions, int32_t *shipped, hipStream_t st);
} // namespace pk

using namespace pk;

namespace {

thread_local std::string g_err;

pk_status fail(pk_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t _e = (expr);                                                              \
        if (_e != hipSuccess)                                                                \
            return fail(PK_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(_e));          \
    } while (0)

constexpr int DEFAULT_BLOCK_GREEDY = 1024;
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
    p.seg_key = c.take<int32_t>(s.n_seg_max);
    p.seg_sr0 = c.take<int32_t>(s.n_seg_max + 1);
    p.split_segs = c.take<int32_t>(s.n_seg_max);
    p.fr[0] = c.take<int32_t>(s.n_seg_max);
    p.fr[1] = c.take<int32_t>(s.n_seg_max);
    p.split_list = c.take<int32_t>(s.n_split_max);
    p.u = c.take<int32_t>(s.n_split_max * d.N);
    p.E = c.take<int32_t>(s.n_split_max * d.N);
    p.rank = c.take<int16_t>((int64_t)d.n_traj * d.R * d.N);
    *setup_scratch = c.take<char>((int64_t)setup_scratch_bytes(d.total));
    if (L) *L = p;
}

size_t serial_bytes(const Dims &d)
{
    Carver c{nullptr};
    c.take<int64_t>(d.n_traj + 1);
    c.take<int16_t>((int64_t)d.n_traj * d.R * d.N);
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

} // namespace

extern "C" {

const char *pk_last_error(void) { return g_err.c_str(); }

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
    *bytes = std::max(picard_bytes(d, policy, B), serial_bytes(d));
    return PK_OK;
}

pk_status pk_serial_simulate(const pk_problem *problem, const pk_policy *policy, void *ws,
                             size_t ws_bytes, int32_t *actions, int32_t *shipped,
                             int32_t *final_inv, int32_t validate, void *stream)
{
    g_err.clear();
    Dims d;
    pk_status s = check_problem(problem, &d);
    if (s != PK_OK) return s;
    if ((s = check_policy(policy)) != PK_OK) return s;
    if (d.total > 0 && !actions) return fail(PK_ERR_INVALID_ARG, "actions is NULL");
    if (policy->kind != PK_POLICY_GREEDY)
        return fail(PK_ERR_UNSUPPORTED, "serial learned policy not built yet");
    if (!ws || ws_bytes < serial_bytes(d)) return fail(PK_ERR_WORKSPACE, "workspace too small");
    hipStream_t st = (hipStream_t)stream;
    Carver c{align_ws(ws)};
    int64_t *to = c.take<int64_t>(d.n_traj + 1);
    int16_t *rank = c.take<int16_t>((int64_t)d.n_traj * d.R * d.N);
    int32_t *state = final_inv ? final_inv : c.take<int32_t>((int64_t)d.n_traj * d.K * d.N);
    HIP_TRY(hipMemcpyAsync(to, problem->traj_offsets, (d.n_traj + 1) * sizeof(int64_t),
                           hipMemcpyHostToDevice, st));
    Prob P = make_prob(problem, d, to);
    HIP_TRY(hipMemcpyAsync(state, problem->init_inv, (size_t)d.n_traj * d.K * d.N * 4,
                           hipMemcpyDeviceToDevice, st));
    HIP_TRY(setup_rank(P, rank, st));
    (void)validate;
    HIP_TRY(launch_serial_greedy(P, rank, state, actions, shipped, st));
    HIP_TRY(hipStreamSynchronize(st));
    return PK_OK;
}

pk_status pk_picard_simulate(const pk_problem *problem, const pk_policy *policy,
                             const pk_picard_opts *opts, void *ws, size_t ws_bytes,
                             int32_t *actions, int32_t *shipped, int32_t *final_inv,
                             pk_stats *stats, void *stream)
{
    g_err.clear();
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
    if (policy->kind != PK_POLICY_GREEDY)
        return fail(PK_ERR_UNSUPPORTED, "learned-policy Picard not built yet");
    const int B = o.block_len > 0 ? o.block_len : DEFAULT_BLOCK_GREEDY;
    const int64_t mp64 = o.max_passes > 0 ? o.max_passes : d.max_T + 1;
    const int max_passes = (int)std::min<int64_t>(mp64, 0x7ffffff0);
    if (!ws || ws_bytes < picard_bytes(d, policy, B))
        return fail(PK_ERR_WORKSPACE, "workspace too small: need %zu bytes, got %zu",
                    picard_bytes(d, policy, B), ws_bytes);
    if (!o.use_frontier)
        return fail(PK_ERR_UNSUPPORTED, "use_frontier=0 not built yet");
    if (walk_greedy_lds(d.N, d.R) > 65536)
        return fail(PK_ERR_SHAPE, "N=%d, R=%d need more LDS than a workgroup has", d.N, d.R);
    hipStream_t st = (hipStream_t)stream;
    Carver c{align_ws(ws)};
    Plan L;
    int64_t *to;
    void *scratch;
    carve_plan(c, d, policy, B, &L, &to, &scratch);
    const Sizes sz = plan_sizes(d, B);
    HIP_TRY(hipMemcpyAsync(to, problem->traj_offsets, (d.n_traj + 1) * sizeof(int64_t),
                           hipMemcpyHostToDevice, st));
    Prob P = make_prob(problem, d, to);
    HIP_TRY(setup_ctl(L, d.n_traj, max_passes, st));
    const bool has_init = o.init_cache != nullptr;
    if (d.total > 0) {
        HIP_TRY(setup_plan(P, L, o.init_cache, o.validate, false, (int32_t)sz.n_seg_max, scratch,
                           st));
        HIP_TRY(setup_rank(P, L.rank, st));
        if (has_init) HIP_TRY(launch_consume(P, L, sz.n_split_max, st));
    }
    if (final_inv)
        HIP_TRY(hipMemcpyAsync(final_inv, problem->init_inv, (size_t)d.n_traj * d.K * d.N * 4,
                               hipMemcpyDeviceToDevice, st));
    Ctl *hc = g_pinned.get();
    if (!hc) return fail(PK_ERR_HIP, "pinned host allocation failed");
    const int grid = num_cus() * 8;
    const int U = o.graph_unroll > 0 ? o.graph_unroll : 8;
    const bool timing = stats && stats->timing;
    std::vector<hipEvent_t> evs;
    int launched = 0;
    int done = 0;
    if (d.total == 0) {
        done = 1;
    }
    while (!done && launched < max_passes) {
        const int u = std::min(U, max_passes - launched);
        for (int i = 0; i < u; ++i) {
            HIP_TRY(launch_scan_entry(P, L, (int)sz.n_seg_max, !has_init, st));
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (timing) {
                HIP_TRY(hipEventCreate(&e0));
                HIP_TRY(hipEventCreate(&e1));
                HIP_TRY(hipEventRecord(e0, st));
            }
            HIP_TRY(launch_walk_greedy(P, L, final_inv, has_init, grid, st));
            if (timing) {
                HIP_TRY(hipEventRecord(e1, st));
                evs.push_back(e0);
                evs.push_back(e1);
            }
            HIP_TRY(launch_pass_end(L, st));
        }
        launched += u;
        HIP_TRY(hipMemcpyAsync(hc, L.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        done = hc->done;
    }
    if (d.total > 0) HIP_TRY(launch_unpermute(P, L, actions, shipped, st));
    HIP_TRY(hipMemcpyAsync(hc, L.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    std::vector<int32_t> lcp(d.n_traj);
    HIP_TRY(hipMemcpyAsync(lcp.data(), L.traj_lcp, d.n_traj * sizeof(int32_t),
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (stats) {
        if (stats->passes)
            for (int b = 0; b < d.n_traj; ++b) stats->passes[b] = lcp[b] + 1;
        stats->passes_max = d.total > 0 ? hc->passes_done : 1;
        stats->block_len = B;
        stats->changed_total = (int64_t)hc->changed_total;
        stats->runs_walked = (int64_t)hc->runs_walked;
        stats->orders_walked = (int64_t)hc->orders_walked;
        stats->near_ties = (int64_t)hc->near_ties;
        stats->walk_bytes = (int64_t)hc->bytes_walked;
        stats->walk_ms = 0.0;
        stats->walk_launches = (int64_t)(evs.size() / 2);
        for (size_t i = 0; i + 1 < evs.size(); i += 2) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, evs[i], evs[i + 1]) == hipSuccess) stats->walk_ms += ms;
        }
    }
    for (hipEvent_t e : evs) (void)hipEventDestroy(e);
    if (hc->error) return fail(PK_ERR_INVALID_ARG, "input value out of range (code %d)", hc->error);
    if (d.total > 0 && hc->done != 1)
        return fail(PK_ERR_NOT_CONVERGED, "not converged after %d passes", hc->passes_done);
    return PK_OK;
}

pk_status pk_policy_grad(const pk_problem *problem, const pk_policy *policy,
                         const int32_t *actions, const float *advantages, float *logp,
                         float *grad, double *objective, void *ws, size_t ws_bytes,
                         int32_t validate, void *stream)
{
    g_err.clear();
    (void)problem; (void)policy; (void)actions; (void)advantages; (void)logp; (void)grad;
    (void)objective; (void)ws; (void)ws_bytes; (void)validate; (void)stream;
    return fail(PK_ERR_UNSUPPORTED, "policy gradient not built yet");
}

pk_status pk_autotune(const pk_problem *problem, const pk_policy *policy, void *ws,
                      size_t ws_bytes, int32_t *best_block_len, void *stream)
{
    g_err.clear();
    (void)problem; (void)policy; (void)ws; (void)ws_bytes; (void)stream;
    if (best_block_len) *best_block_len = DEFAULT_BLOCK_GREEDY;
    return fail(PK_ERR_UNSUPPORTED, "autotune not built yet");
}

} // extern "C"

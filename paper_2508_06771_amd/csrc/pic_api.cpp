// pic_api.cpp -- the C ABI: context, argument checks, scratch management and
// the order of launches of one collision step.
#include <math.h>
#include <string.h>

#include <stdio.h>
#include <stdlib.h>

#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "pic_internal.hpp"

// Scratch of coulomb_collide_noalloc: a fixed array in the code object, one
// copy per GPU.  Host code uses only the per-device address that
// hipGetSymbolAddress returns (the array's name is a host-side stand-in).
static __device__ __align__(256) unsigned char scratch[PIC_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// The address of this GPU's copy of `scratch`, taken once per device with the
// device current (the caller has set it).
void *noalloc_scratch(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch_ptr[device] = p;
    }
    return g_scratch_ptr[device];
}
}  // namespace

struct pic_ctx {
    int device = 0;
    void *noalloc = nullptr;   // this device's copy of `scratch`
    hipStream_t stream = nullptr;
    int num_cu = 256;
    size_t lds_max = 65536;
    DevFlags *flags = nullptr;
    void *ws = nullptr;
    size_t ws_cap = 0;
    size_t ws_limit = 0;   // most scratch bytes the context may hold (0: no limit)
    double mcc_sigma0 = 0.0, mcc_nn = 0.0, mcc_mr = 0.0;
    // DSMC-Coll cross-section table (device copy) and its host header
    double *dsmc_buf = nullptr;
    DsmcTable dsmc_tab = {0, nullptr, nullptr, {0, 0, 0, 0}, 0.0};
    bool mcc_set = false;
    double *moments_out = nullptr;
    // graph of one steady-state step (pic_run_steps)
    uint64_t *step_dev = nullptr;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t exec = nullptr;
    unsigned char graph_key[512];
    size_t graph_key_len = 0;
    // learned gate
    const float *gate_params = nullptr;
    float gate_thr = 0.5f;
    int gate_kmax = 8;
    double gate_judge_frac = 0.01, gate_tol = 1e-3, gate_max_false = 0.1;
    int gate_mom_every = 1;
    int gate_replicas = 8, gate_bf16 = 1, gate_analytic = 0;
    void *mlp_w = nullptr;   // mlp_train_step: parameters of the previous call, its step count
    int32_t mlp_t = 0;
    uint32_t gate_min_judged = 20;
    DevGate *gate_dev = nullptr;
    int32_t gate_M = 0;
    void *gate_mem = nullptr;
    double *gate_mom = nullptr, *gate_dts = nullptr, *gate_r = nullptr;
    int32_t *gate_k = nullptr, *gate_judge = nullptr;
    uint8_t *gate_skip = nullptr, *gate_want = nullptr;
    float *gate_prob = nullptr;
    // per-cell conservation debt (PIC_CONSERVE_FIX)
    double *debt = nullptr;
    int32_t debt_M = 0;
    // autotuned class thresholds / grid sizes per dtype
    ClassCaps tuned[2];
    bool tuned_valid[2] = {false, false};
};

namespace {

struct TimedLaunch {
    int slot;
    hipEvent_t beg, end;
};
// The context whose launches are being timed (calls on one context are issued
// from one host thread).
struct Timing {
    bool on = false;
    std::vector<TimedLaunch> open;
};
Timing g_timing;

}  // namespace

void ktime_begin(int slot, hipStream_t st)
{
    if (!g_timing.on) return;
    TimedLaunch t;
    t.slot = slot;
    if (hipEventCreate(&t.beg) != hipSuccess || hipEventCreate(&t.end) != hipSuccess) return;
    (void)hipEventRecord(t.beg, st);
    g_timing.open.push_back(t);
}

bool ktime_pause()
{
    const bool was = g_timing.on;
    g_timing.on = false;
    return was;
}

void ktime_resume(bool was) { g_timing.on = was; }

void ktime_end(int slot, hipStream_t st)
{
    if (!g_timing.on) return;
    for (auto it = g_timing.open.rbegin(); it != g_timing.open.rend(); ++it)
        if (it->slot == slot) {
            (void)hipEventRecord(it->end, st);
            return;
        }
}

namespace {

#define CK(x)                                   \
    do {                                        \
        if ((x) != hipSuccess) return PIC_ERR_HIP; \
    } while (0)
#define RC(x)                         \
    do {                              \
        int rc_ = (x);                \
        if (rc_ != PIC_OK) return rc_; \
    } while (0)

struct Bump {
    unsigned char *p;
    size_t used = 0;
    explicit Bump(void *base) : p((unsigned char *)base) {}
    void *take(size_t bytes)
    {
        void *r = p + used;
        used += (bytes + 255) & ~(size_t)255;
        return r;
    }
};

int ensure_ws(pic_ctx *c, size_t bytes)
{
    if (bytes <= c->ws_cap) return PIC_OK;
    if (c->ws_limit && bytes > c->ws_limit) return PIC_ERR_NOMEM;   // beyond the caller's budget
    CK(hipSetDevice(c->device));
    CK(hipStreamSynchronize(c->stream));
    if (c->ws) {
        CK(hipFree(c->ws));
        c->ws = nullptr;
        c->ws_cap = 0;
    }
    size_t want = bytes + bytes / 8;
    if (c->ws_limit && want > c->ws_limit) want = c->ws_limit;
    if (hipMalloc(&c->ws, want) != hipSuccess) {
        (void)hipGetLastError();
        c->ws = nullptr;
        return PIC_ERR_NOMEM;
    }
    c->ws_cap = want;
    return PIC_OK;
}

// Per-cell gate state for n_cells cells (allocated outside any capture).
int ensure_gate(pic_ctx *c, int32_t M)
{
    if (c->gate_M == M && c->gate_mem) return PIC_OK;
    CK(hipSetDevice(c->device));
    CK(hipStreamSynchronize(c->stream));
    if (c->gate_mem) CK(hipFree(c->gate_mem));
    c->gate_mem = nullptr;
    c->gate_M = 0;
    const size_t m = (size_t)M;
    const size_t bytes = m * (14 * 8 + 8 + 8 + 4 + 4 + 1 + 1 + 4) + 8 * 256;
    if (hipMalloc(&c->gate_mem, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return PIC_ERR_NOMEM;
    }
    Bump b(c->gate_mem);
    c->gate_mom = (double *)b.take(m * 14 * 8);
    c->gate_dts = (double *)b.take(m * 8);
    c->gate_r = (double *)b.take(m * 8);
    c->gate_k = (int32_t *)b.take(m * 4);
    c->gate_judge = (int32_t *)b.take(m * 4);
    c->gate_skip = (uint8_t *)b.take(m);
    c->gate_want = (uint8_t *)b.take(m);
    c->gate_prob = (float *)b.take(m * 4);
    CK(hipMemset(c->gate_mem, 0, bytes));
    CK(hipMemset(c->gate_dev, 0, sizeof(DevGate)));
    CK(hipDeviceSynchronize());
    c->gate_M = M;
    return PIC_OK;
}

int ensure_debt(pic_ctx *c, int32_t M)
{
    if (c->debt_M == M && c->debt) return PIC_OK;
    CK(hipSetDevice(c->device));
    CK(hipStreamSynchronize(c->stream));
    if (c->debt) CK(hipFree(c->debt));
    c->debt = nullptr;
    c->debt_M = 0;
    if (hipMalloc((void **)&c->debt, (size_t)M * 4 * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return PIC_ERR_NOMEM;
    }
    CK(hipMemset(c->debt, 0, (size_t)M * 4 * sizeof(double)));
    CK(hipDeviceSynchronize());
    c->debt_M = M;
    return PIC_OK;
}

int ceil_log2(int64_t x)
{
    int b = 0;
    while (((int64_t)1 << b) < x) ++b;
    return b;
}

// Null-collision threshold floor(P_null 2^32), P_null = 1 - exp(-nu_max dt),
// nu_max = n_n sigma0 sqrt(2) (sigma = sigma0 E^-1/2, E = |v|^2 / 2).
uint64_t mcc_threshold(double dt, double sigma0, double n_neutral)
{
    const double nu_max = n_neutral * sigma0 * sqrt(2.0);
    const double p = 1.0 - exp(-nu_max * dt);
    double t = floor(p * 4294967296.0);
    if (t < 0.0) t = 0.0;
    if (t > 4294967296.0) t = 4294967296.0;
    return (uint64_t)t;
}

// Stable LSD passes by cell id over the given streams, an even number of
// passes so the result ends where it started.  cur_* are the caller's arrays.
struct SortStreams {
    int32_t *key;
    int n32;
    uint32_t *p32[5];
    int n64;
    uint64_t *p64[3];
};

int sort_by_cell(hipStream_t st, const SortStreams &caller, const SortStreams &tmp, int64_t n,
                 int32_t n_cells, const BinScratch &bs, const int *gate)
{
    const int bits = ceil_log2(n_cells);
    if (bits == 0 || n <= 1) return PIC_OK;
    const int passes = 2 * ((bits + 15) / 16);
    const int per = (bits + passes - 1) / passes;
    for (int ps = 0; ps < passes; ++ps) {
        const SortStreams &src = (ps % 2 == 0) ? caller : tmp;
        const SortStreams &dst = (ps % 2 == 0) ? tmp : caller;
        RadixPass p;
        memset(&p, 0, sizeof(p));
        p.key_in = src.key;
        p.key_out = dst.key;
        p.n32 = src.n32;
        for (int s = 0; s < src.n32; ++s) {
            p.p32_in[s] = src.p32[s];
            p.p32_out[s] = dst.p32[s];
        }
        p.n64 = src.n64;
        for (int s = 0; s < src.n64; ++s) {
            p.p64_in[s] = src.p64[s];
            p.p64_out[s] = dst.p64[s];
        }
        p.iota_slot = -1;
        p.n = n;
        p.shift = ps * per;
        p.bits = per;
        if (p.shift + p.bits > bits) p.bits = bits - p.shift;
        if (p.bits <= 0) p.bits = 1;
        p.gate = gate;
        RC(radix_pass(p, bs, st));
    }
    return PIC_OK;
}

int check_dtype(int dtype) { return (dtype == PIC_F32 || dtype == PIC_F64) ? PIC_OK : PIC_ERR_DTYPE; }

}  // namespace

extern "C" {

const char *pic_strerror(int s)
{
    switch (s) {
    case PIC_OK: return "ok";
    case PIC_ERR_ARG: return "invalid argument";
    case PIC_ERR_RANGE: return "cell id out of range";
    case PIC_ERR_NONFINITE: return "non-finite velocity after the step";
    case PIC_ERR_HIP: return "HIP runtime error";
    case PIC_ERR_NOMEM: return "out of device memory";
    case PIC_ERR_DTYPE: return "unknown dtype";
    case PIC_ERR_STATE: return "invalid state (storage asserted sorted was not)";
    default: return "unknown status";
    }
}

int pic_create(pic_ctx **out, int device, void *hip_stream)
{
    if (!out) return PIC_ERR_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return PIC_ERR_ARG;
    pic_ctx *c = new (std::nothrow) pic_ctx();
    if (!c) return PIC_ERR_NOMEM;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    if (hipSetDevice(device) != hipSuccess) {
        delete c;
        return PIC_ERR_HIP;
    }
    c->noalloc = noalloc_scratch(device);   // null: coulomb_collide_noalloc reports PIC_ERR_STATE
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && v > 0)
        c->num_cu = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && v > 0)
        c->lds_max = (size_t)v;
    if (hipMalloc((void **)&c->flags, sizeof(DevFlags)) != hipSuccess) {
        delete c;
        return PIC_ERR_NOMEM;
    }
    if (hipMalloc((void **)&c->gate_dev, sizeof(DevGate)) != hipSuccess ||
        hipMemset(c->gate_dev, 0, sizeof(DevGate)) != hipSuccess) {
        (void)hipFree(c->flags);
        delete c;
        return PIC_ERR_NOMEM;
    }
    if (hipMalloc((void **)&c->step_dev, 256) != hipSuccess) {
        (void)hipFree(c->flags);
        delete c;
        return PIC_ERR_NOMEM;
    }
    if (hipMemset(c->flags, 0, sizeof(DevFlags)) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(c->flags);
        (void)hipFree(c->step_dev);
        delete c;
        return PIC_ERR_HIP;
    }
    *out = c;
    return PIC_OK;
}

void pic_destroy(pic_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (c->exec) (void)hipGraphExecDestroy(c->exec);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->ws) (void)hipFree(c->ws);
    if (c->flags) (void)hipFree(c->flags);
    if (c->step_dev) (void)hipFree(c->step_dev);
    if (c->gate_dev) (void)hipFree(c->gate_dev);
    if (c->gate_mem) (void)hipFree(c->gate_mem);
    if (c->debt) (void)hipFree(c->debt);
    if (c->dsmc_buf) (void)hipFree(c->dsmc_buf);
    delete c;
}

int pic_set_stream(pic_ctx *c, void *hip_stream)
{
    if (!c) return PIC_ERR_ARG;
    c->stream = (hipStream_t)hip_stream;
    return PIC_OK;
}

int pic_sync(pic_ctx *c)
{
    if (!c) return PIC_ERR_ARG;
    CK(hipSetDevice(c->device));
    CK(hipStreamSynchronize(c->stream));
    int host[5] = {0, 0, 0, 0, 0};
    CK(hipMemcpy(host, c->flags, sizeof(host), hipMemcpyDeviceToHost));
    if (host[2] || host[3] || host[4]) {
        const int zero[3] = {0, 0, 0};
        CK(hipMemcpy(&c->flags->sticky_range, zero, sizeof(zero), hipMemcpyHostToDevice));
    }
    if (host[2]) return PIC_ERR_RANGE;
    if (host[3]) return PIC_ERR_STATE;
    if (host[4]) return PIC_ERR_NONFINITE;
    return PIC_OK;
}

int pic_set_mcc(pic_ctx *c, double sigma0, double n_neutral, double mass_ratio)
{
    if (!c || !(sigma0 >= 0.0) || !(n_neutral >= 0.0) || !(mass_ratio >= 0.0) || !(mass_ratio < 0.5))
        return PIC_ERR_ARG;
    c->mcc_sigma0 = sigma0;
    c->mcc_nn = n_neutral;
    c->mcc_mr = mass_ratio;
    c->mcc_set = true;
    return PIC_OK;
}

int pic_set_dsmc(pic_ctx *c, int32_t nseg, const double *breaks, const double *coef,
                 const double *threshold, double mass_ratio)
{
    if (!c || nseg < 1 || nseg > DSMC_MAX_SEG || !breaks || !coef || !threshold ||
        !(mass_ratio >= 0.0) || !(mass_ratio < 0.5) || breaks[0] != 0.0)
        return PIC_ERR_ARG;
    for (int32_t p = 0; p < nseg; ++p)
        if (!(breaks[p + 1] > breaks[p])) return PIC_ERR_ARG;
    for (int k = 0; k < 4; ++k)
        if (!(threshold[k] >= 0.0)) return PIC_ERR_ARG;
    CK(hipSetDevice(c->device));
    const size_t nb = (size_t)(nseg + 1) + (size_t)4 * nseg * 4;
    std::vector<double> host(nb);
    memcpy(host.data(), breaks, (size_t)(nseg + 1) * sizeof(double));
    memcpy(host.data() + nseg + 1, coef, (size_t)4 * nseg * 4 * sizeof(double));
    CK(hipStreamSynchronize(c->stream));
    if (c->dsmc_buf) CK(hipFree(c->dsmc_buf));
    c->dsmc_buf = nullptr;
    if (hipMalloc((void **)&c->dsmc_buf, nb * sizeof(double)) != hipSuccess) return PIC_ERR_NOMEM;
    CK(hipMemcpy(c->dsmc_buf, host.data(), nb * sizeof(double), hipMemcpyHostToDevice));
    c->dsmc_tab.nseg = nseg;
    c->dsmc_tab.breaks = c->dsmc_buf;
    c->dsmc_tab.coef = c->dsmc_buf + nseg + 1;
    for (int k = 0; k < 4; ++k) c->dsmc_tab.thr[k] = threshold[k];
    c->dsmc_tab.mass_ratio = mass_ratio;
    return PIC_OK;
}

int dsmc_collide(pic_ctx *c, int dtype, void *v, const int32_t *cell_of, const uint32_t *pid,
                 int64_t n, int32_t n_cells, const double *n_gas, const double *n_meta, double n_gas0,
                 double n_meta0, double dt, uint64_t seed, uint64_t step, uint32_t pid_base,
                 void *v_new, uint32_t *pid_new, int32_t *cell_new, int64_t cap, uint64_t *count,
                 uint8_t *channel_out)
{
    if (!c || n < 0 || n_cells < 1 || cap < 0 || !count || !(dt > 0.0) || !(n_gas0 >= 0.0) ||
        !(n_meta0 >= 0.0))
        return PIC_ERR_ARG;
    if (n > 0 && (!v || !cell_of || !pid)) return PIC_ERR_ARG;
    if (cap > 0 && (!v_new || !pid_new || !cell_new)) return PIC_ERR_ARG;
    RC(check_dtype(dtype));
    if (!c->dsmc_buf) return PIC_ERR_STATE;
    CK(hipSetDevice(c->device));
    DsmcArgs a;
    memset(&a, 0, sizeof(a));
    a.v = v;
    a.n = n;
    a.n_cells = n_cells;
    a.cell = cell_of;
    a.pid = pid;
    a.ng = n_gas;
    a.nm = n_meta;
    a.ng0 = n_gas0;
    a.nm0 = n_meta0;
    a.dt = dt;
    a.seed = seed;
    a.step = step;
    a.pid_base = pid_base;
    a.v_new = v_new;
    a.cap = cap;
    a.pid_new = pid_new;
    a.cell_new = cell_new;
    a.count = (unsigned long long *)count;
    a.chan_out = channel_out;
    a.dflags = c->flags;
    ktime_begin(KT_DSMC, c->stream);
    const int rc = launch_dsmc(dtype, a, c->dsmc_tab, c->stream);
    ktime_end(KT_DSMC, c->stream);
    return rc;
}

int pic_time_kernels(pic_ctx *c, int on)
{
    if (!c) return PIC_ERR_ARG;
    g_timing.on = on != 0;
    return PIC_OK;
}

int pic_kernel_times(pic_ctx *c, double *ms, int64_t *count)
{
    if (!c || !ms || !count) return PIC_ERR_ARG;
    CK(hipSetDevice(c->device));
    for (int s = 0; s < KT_SLOTS; ++s) {
        ms[s] = 0.0;
        count[s] = 0;
    }
    for (auto &t : g_timing.open) {
        float e = 0.0f;
        if (hipEventSynchronize(t.end) == hipSuccess && hipEventElapsedTime(&e, t.beg, t.end) == hipSuccess &&
            t.slot >= 0 && t.slot < KT_SLOTS) {
            ms[t.slot] += e;
            count[t.slot] += 1;
        }
        (void)hipEventDestroy(t.beg);
        (void)hipEventDestroy(t.end);
    }
    g_timing.open.clear();
    return PIC_OK;
}

int pic_set_moments_out(pic_ctx *c, double *out)
{
    if (!c) return PIC_ERR_ARG;
    c->moments_out = out;
    return PIC_OK;
}

int pic_conserve_reset(pic_ctx *c)
{
    if (!c) return PIC_ERR_ARG;
    if (!c->debt) return PIC_OK;
    CK(hipSetDevice(c->device));
    CK(hipStreamSynchronize(c->stream));
    CK(hipMemset(c->debt, 0, (size_t)c->debt_M * 4 * sizeof(double)));
    CK(hipDeviceSynchronize());
    return PIC_OK;
}

int pic_gate_config(pic_ctx *c, const float *params, float threshold, int32_t k_max,
                    double judge_fraction, double tolerance, int32_t replicas, int bf16)
{
    if (!c || !params || !(threshold >= 0.0f) || k_max < 0 || !(judge_fraction >= 0.0) ||
        !(judge_fraction <= 1.0) || !(tolerance > 0.0) || replicas < 1)
        return PIC_ERR_ARG;
    c->gate_params = params;
    c->gate_analytic = 0;
    c->gate_thr = threshold;
    c->gate_kmax = k_max;
    c->gate_judge_frac = judge_fraction;
    c->gate_tol = tolerance;
    c->gate_replicas = replicas;
    c->gate_bf16 = bf16 != 0;
    return PIC_OK;
}

int pic_gate_config_analytic(pic_ctx *c, float threshold, int32_t k_max, double judge_fraction,
                             double tolerance, int32_t replicas)
{
    if (!c || !(threshold >= 0.0f) || k_max < 0 || !(judge_fraction >= 0.0) || !(judge_fraction <= 1.0) ||
        !(tolerance > 0.0) || replicas < 1)
        return PIC_ERR_ARG;
    c->gate_params = nullptr;
    c->gate_analytic = 1;
    c->gate_thr = threshold;
    c->gate_kmax = k_max;
    c->gate_judge_frac = judge_fraction;
    c->gate_tol = tolerance;
    c->gate_replicas = replicas;
    return PIC_OK;
}

int pic_analytic_relaxation(pic_ctx *c, const double *moments, int32_t n_cells, double dt, double lnLambda,
                            const double *density, int32_t replicas, double *r_out)
{
    if (!c || !moments || !r_out || n_cells < 1 || !(dt > 0.0) || !(lnLambda > 0.0) || replicas < 1)
        return PIC_ERR_ARG;
    CK(hipSetDevice(c->device));
    return launch_analytic_relax(moments, n_cells, dt, lnLambda, density, replicas, r_out, c->stream);
}

int pic_gate_refresh(pic_ctx *c, int32_t every)
{
    if (!c || every < 1) return PIC_ERR_ARG;
    c->gate_mom_every = every;
    return PIC_OK;
}

int pic_gate_reset(pic_ctx *c)
{
    if (!c) return PIC_ERR_ARG;
    CK(hipSetDevice(c->device));
    CK(hipStreamSynchronize(c->stream));
    CK(hipMemset(c->gate_dev, 0, sizeof(DevGate)));
    if (c->gate_mem && c->gate_M > 0) CK(hipMemset(c->gate_k, 0, (size_t)c->gate_M * 4));
    CK(hipDeviceSynchronize());
    return PIC_OK;
}

int pic_gate_stats(pic_ctx *c, int64_t *out)
{
    if (!c || !out) return PIC_ERR_ARG;
    CK(hipSetDevice(c->device));
    CK(hipStreamSynchronize(c->stream));
    DevGate g;
    CK(hipMemcpy(&g, c->gate_dev, sizeof(g), hipMemcpyDeviceToHost));
    out[0] = (int64_t)g.steps;
    out[1] = (int64_t)g.skipped;
    out[2] = (int64_t)g.collided;
    out[3] = (int64_t)g.judged;
    out[4] = (int64_t)g.judged_want;
    out[5] = (int64_t)g.false_skip;
    out[6] = g.disabled;
    out[7] = g.have_moments;
    return PIC_OK;
}

int pic_gate_state(pic_ctx *c, uint8_t *skip, int32_t *k_acc, float *prob, double *moments)
{
    if (!c) return PIC_ERR_ARG;
    if (!c->gate_mem) return PIC_ERR_STATE;
    CK(hipSetDevice(c->device));
    const size_t M = (size_t)c->gate_M;
    if (skip) CK(hipMemcpyAsync(skip, c->gate_skip, M, hipMemcpyDeviceToDevice, c->stream));
    if (k_acc) CK(hipMemcpyAsync(k_acc, c->gate_k, M * 4, hipMemcpyDeviceToDevice, c->stream));
    if (prob) CK(hipMemcpyAsync(prob, c->gate_prob, M * 4, hipMemcpyDeviceToDevice, c->stream));
    if (moments) CK(hipMemcpyAsync(moments, c->gate_mom, M * 14 * 8, hipMemcpyDeviceToDevice, c->stream));
    return PIC_OK;
}

int pic_features(pic_ctx *c, const double *moments, int32_t n_cells, float *feat, uint8_t *valid)
{
    if (!c || !moments || !feat || n_cells < 1) return PIC_ERR_ARG;
    CK(hipSetDevice(c->device));
    return launch_features(moments, n_cells, feat, valid, c->stream);
}

int pic_relaxation(pic_ctx *c, int dtype, const void *v, int64_t n, const int32_t *cell_start,
                   const uint32_t *pid, int32_t n_cells, double dt, double lnLambda,
                   const double *density, const double *dt_scale, uint64_t seed, uint64_t step,
                   int32_t replicas, double *r_out)
{
    if (!c || n < 0 || n_cells < 1 || !cell_start || !r_out || replicas < 1 || !(dt > 0.0) ||
        !(lnLambda > 0.0) || (n > 0 && (!v || !pid)))
        return PIC_ERR_ARG;
    RC(check_dtype(dtype));
    CK(hipSetDevice(c->device));
    const size_t hb = huge_scratch_bytes(dtype, n);
    RC(ensure_ws(c, hb + relax_part_bytes(n_cells, replicas) + 2048));
    Bump b(c->ws);
    set_huge_scratch(dtype, n, b.take(hb));
    RelaxArgs r;
    memset(&r, 0, sizeof(r));
    r.part = (double *)b.take(relax_part_bytes(n_cells, replicas));
    r.v = v;
    r.n = n;
    r.cell_start = cell_start;
    r.pid = pid;
    r.density = density;
    r.dt_scale = dt_scale;
    r.dt = dt;
    r.lnL = lnLambda;
    r.seed = seed;
    r.step = step;
    r.replicas = replicas;
    r.count = n_cells;
    r.cap = n_cells;
    r.r_out = r_out;
    return launch_relax(dtype, r, c->num_cu, c->stream);
}

int pic_mlp_forward(pic_ctx *c, const float *params, const float *x, int32_t batch, int bf16,
                    float *prob)
{
    if (!c || !params || batch < 0 || (batch > 0 && (!x || !prob))) return PIC_ERR_ARG;
    CK(hipSetDevice(c->device));
    return launch_mlp_forward(params, x, batch, bf16 != 0, prob, c->stream);
}

int gate_infer(pic_ctx *c, const float *feat, int32_t n_cells, const float *params, float threshold,
               int32_t k_max, int bf16, uint8_t *skip, int32_t *k_acc, float *prob_out)
{
    if (!c || n_cells < 0 || k_max < 0 || !(threshold >= 0.0f) ||
        (n_cells > 0 && (!feat || !params || !skip || !k_acc)))
        return PIC_ERR_ARG;
    if (n_cells == 0) return PIC_OK;
    CK(hipSetDevice(c->device));
    float *prob = prob_out;
    if (!prob) {
        RC(ensure_ws(c, (size_t)n_cells * 4 + 256));
        prob = (float *)c->ws;
    }
    RC(launch_mlp_forward(params, feat, n_cells, bf16 != 0, prob, c->stream));
    return launch_gate_infer_decide(prob, n_cells, threshold, k_max, skip, k_acc, c->stream);
}

int pic_mlp_grad(pic_ctx *c, const float *params, const float *x, const float *y, int32_t batch,
                 int bf16, float *grad, float *loss)
{
    if (!c || !params || batch < 1 || !x || !y || !grad) return PIC_ERR_ARG;
    CK(hipSetDevice(c->device));
    RC(ensure_ws(c, mlp_grad_scratch_floats(batch) * 4 + 1024));
    return launch_mlp_grad(params, x, y, batch, bf16 != 0, (float *)c->ws, grad, loss, c->stream);
}

int pic_mlp_train_step(pic_ctx *c, float *params, float *adam_m, float *adam_v, int32_t t, float lr,
                       const float *x, const float *y, int32_t batch, int bf16, float *loss)
{
    if (!c || !params || !adam_m || !adam_v || t < 1 || !(lr > 0.0f) || batch < 1 || !x || !y)
        return PIC_ERR_ARG;
    CK(hipSetDevice(c->device));
    const size_t sf = mlp_grad_scratch_floats(batch);
    RC(ensure_ws(c, (sf + 4801 + 64) * 4 + 1024));
    float *scratch = (float *)c->ws;
    float *grad = scratch + sf;
    RC(launch_mlp_grad(params, x, y, batch, bf16 != 0, scratch, grad, loss, c->stream));
    return launch_adam(params, adam_m, adam_v, grad, t, lr, c->stream);
}

int mlp_train_step(pic_ctx *c, const void *feat, const float *label, int32_t batch, void *w_master,
                   void *adam_state, float lr, float *loss_out)
{
    if (!c || !w_master || !adam_state) return PIC_ERR_ARG;
    const int32_t t = (w_master == c->mlp_w && c->mlp_t < INT32_MAX) ? c->mlp_t + 1 : 1;
    float *m = (float *)adam_state;
    const int rc = pic_mlp_train_step(c, (float *)w_master, m, m + 4801, t, lr, (const float *)feat,
                                      label, batch, 1, loss_out);
    if (rc == PIC_OK) {
        c->mlp_w = w_master;
        c->mlp_t = t;
    }
    return rc;
}

int pic_bin_cells(pic_ctx *c, const int32_t *cell_of, int64_t n, int32_t n_cells,
                  int32_t *cell_start, int32_t *order)
{
    if (!c || n < 0 || n > INT32_MAX || n_cells < 1 || n_cells > (1 << 24) || !cell_start)
        return PIC_ERR_ARG;
    if (n > 0 && (!cell_of || !order)) return PIC_ERR_ARG;
    CK(hipSetDevice(c->device));
    const size_t need = 4 * (size_t)n * 4 + radix_scratch_bytes(n) + 4096;
    RC(ensure_ws(c, need));
    Bump b(c->ws);
    int32_t *kA = (int32_t *)b.take(4 * (size_t)n);
    int32_t *kB = (int32_t *)b.take(4 * (size_t)n);
    uint32_t *iA = (uint32_t *)b.take(4 * (size_t)n);
    uint32_t *iB = (uint32_t *)b.take(4 * (size_t)n);
    BinScratch bs;
    bs.hist = (uint32_t *)b.take(radix_scratch_bytes(n));
    bs.bsum = bs.hist + 256 * ((n + 4095) / 4096 + 1);   // block sums follow the histogram
    RC(launch_reset_flags(c->flags, c->stream));
    const int bits = ceil_log2(n_cells);
    const int32_t *sorted_keys = cell_of;
    if (n > 0) {
        // pass 0 reads the caller's ids and emits the storage index; an even
        // number of passes, the last writing the index into `order`
        const int passes = bits == 0 ? 0 : 2 * ((bits + 15) / 16);
        const int per = passes ? (bits + passes - 1) / passes : 0;
        if (passes == 0) {
            // single cell: the order is the identity
            RadixPass p;
            memset(&p, 0, sizeof(p));
            p.key_in = cell_of;
            p.key_out = kA;
            p.n32 = 1;
            p.p32_in[0] = nullptr;
            p.p32_out[0] = (uint32_t *)order;
            p.iota_slot = 0;
            p.n = n;
            p.shift = 0;
            p.bits = 1;
            RC(radix_pass(p, bs, c->stream));
            sorted_keys = kA;
        }
        for (int ps = 0; ps < passes; ++ps) {
            RadixPass p;
            memset(&p, 0, sizeof(p));
            p.key_in = ps == 0 ? cell_of : (ps % 2 ? kA : kB);
            p.key_out = ps % 2 ? kB : kA;
            p.n32 = 1;
            p.p32_in[0] = ps == 0 ? nullptr : (ps % 2 ? iA : iB);
            p.p32_out[0] = (ps == passes - 1) ? (uint32_t *)order : (ps % 2 ? iB : iA);
            p.iota_slot = ps == 0 ? 0 : -1;
            p.n = n;
            p.shift = ps * per;
            p.bits = per;
            if (p.shift + p.bits > bits) p.bits = bits - p.shift;
            if (p.bits <= 0) p.bits = 1;
            RC(radix_pass(p, bs, c->stream));
            sorted_keys = p.key_out;
        }
    }
    RC(launch_bin_check(sorted_keys, n, n_cells, cell_start, c->flags, 0, nullptr, c->stream));
    return PIC_OK;
}

struct StepArgs {
    int dtype;
    void *v;
    int32_t *cell_of;
    uint32_t *pid;
    int64_t n;
    int32_t n_cells;
    double dt, lnL;
    const double *density;
    uint64_t seed, step;
    uint32_t flags;
    // bit c: list c (size classes 0..3, 4 = beyond them) may hold cells; a
    // caller that knows the cell sizes clears the empty ones
    uint32_t live = ~0u;
};

static size_t step_ws_bytes(const pic_ctx *c, const StepArgs &s)
{
    const size_t es = s.dtype == PIC_F32 ? 4 : 8;
    const size_t part = (s.flags & PIC_GATE) ? relax_part_bytes(s.n_cells, c->gate_replicas) : 0;
    return (size_t)(s.n_cells + 1) * 4 + (size_t)s.n_cells * (QUEUE_LISTS + 1) * 4 + (size_t)s.n * (8 + 3 * es) +
           radix_scratch_bytes(s.n) + huge_scratch_bytes(s.dtype, s.n) +
           seg_scratch_bytes(s.dtype, s.n, s.n_cells) + part + 8192;
}

static int step_check(pic_ctx *c, const StepArgs &s)
{
    RC(check_dtype(s.dtype));
    if (s.n < 0 || s.n > INT32_MAX || s.n_cells < 1 || s.n_cells > (1 << 24) || !(s.dt > 0.0) ||
        !(s.lnL > 0.0))
        return PIC_ERR_ARG;
    if (s.n > 0 && (!s.v || !s.cell_of || !s.pid)) return PIC_ERR_ARG;
    if ((s.flags & PIC_FUSE_MCC) && !c->mcc_set) return PIC_ERR_STATE;
    if ((s.flags & PIC_MOMENTS) && !(s.flags & PIC_GATE) && !c->moments_out) return PIC_ERR_STATE;
    if ((s.flags & PIC_GATE) && !c->gate_params && !c->gate_analytic) return PIC_ERR_STATE;
    return PIC_OK;
}

// All launches of one step on stream st.  step_dev: step number in device
// memory (graph replays) or NULL (s.step by value).
static int step_enqueue(pic_ctx *c, const StepArgs &s, hipStream_t st, const uint64_t *step_dev)
{
    const int dtype = s.dtype;
    const int64_t n = s.n;
    const int32_t n_cells = s.n_cells;
    const size_t es = dtype == PIC_F32 ? 4 : 8;
    Bump b(c->ws);
    int32_t *cs = (int32_t *)b.take((size_t)(n_cells + 1) * 4);
    int32_t *lists = (int32_t *)b.take((size_t)n_cells * QUEUE_LISTS * 4);
    int32_t *order = (int32_t *)b.take((size_t)n_cells * 4);
    int32_t *tkey = (int32_t *)b.take((size_t)n * 4);
    uint32_t *tpid = (uint32_t *)b.take((size_t)n * 4);
    void *tv = b.take((size_t)n * 3 * es);
    BinScratch bs;
    bs.hist = (uint32_t *)b.take(radix_scratch_bytes(n));
    bs.bsum = bs.hist + 256 * ((n + 4095) / 4096 + 1);
    set_huge_scratch(dtype, n, b.take(huge_scratch_bytes(dtype, n)));
    // the re-binning buffers are free again by the collide pass: the
    // segmented path of the largest cells copies members into them
    set_seg_scratch(dtype, n, n_cells, b.take(seg_scratch_bytes(dtype, n, n_cells)), tkey, tpid, tv);
    double *relax_part = (s.flags & PIC_GATE)
                             ? (double *)b.take(relax_part_bytes(n_cells, c->gate_replicas))
                             : nullptr;

    RC(launch_reset_flags(c->flags, st));
    const bool assume = (s.flags & PIC_ASSUME_SORTED) != 0;
    ktime_begin(KT_CHECK, st);
    RC(launch_bin_check(s.cell_of, n, n_cells, cs, c->flags, assume ? 2 : 1, nullptr, st));
    ktime_end(KT_CHECK, st);
    if (!assume && n > 1 && n_cells > 1) {
        ktime_begin(KT_SORT, st);
        SortStreams caller, tmp;
        memset(&caller, 0, sizeof(caller));
        memset(&tmp, 0, sizeof(tmp));
        caller.key = s.cell_of;
        tmp.key = tkey;
        caller.n32 = tmp.n32 = 1;
        caller.p32[0] = s.pid;
        tmp.p32[0] = tpid;
        if (dtype == PIC_F32) {
            caller.n32 = tmp.n32 = 4;
            for (int k = 0; k < 3; ++k) {
                caller.p32[1 + k] = (uint32_t *)s.v + (size_t)k * n;
                tmp.p32[1 + k] = (uint32_t *)tv + (size_t)k * n;
            }
        } else {
            caller.n64 = tmp.n64 = 3;
            for (int k = 0; k < 3; ++k) {
                caller.p64[k] = (uint64_t *)s.v + (size_t)k * n;
                tmp.p64[k] = (uint64_t *)tv + (size_t)k * n;
            }
        }
        RC(sort_by_cell(st, caller, tmp, n, n_cells, bs, &c->flags->unsorted));
        RC(launch_bin_check(s.cell_of, n, n_cells, cs, c->flags, 0, &c->flags->unsorted, st));
        ktime_end(KT_SORT, st);
    }
    ClassCaps caps = c->tuned_valid[dtype] ? c->tuned[dtype] : collide_caps(dtype, c->lds_max);
    const uint64_t mcc_thr = (s.flags & PIC_FUSE_MCC) ? mcc_threshold(s.dt, c->mcc_sigma0, c->mcc_nn) : 0;
    const bool gate = (s.flags & PIC_GATE) != 0;
    // the plain binary64 step (no correction, no fused moment sums) runs its
    // largest class with the lean pass, which holds cells of up to
    // lean64_cap() members on one workgroup (not with the one-launch schedule)
    if (dtype == PIC_F64 && !caps.unified && !(s.flags & PIC_CONSERVE_FIX) &&
        (gate || !(s.flags & PIC_MOMENTS)) && caps.cap[3] < lean64_cap())
        caps.cap[3] = lean64_cap();
    // cells beyond the LDS classes: several workgroups each, unless the step
    // needs whole-cell sums (conservation correction, fused moments)
    const bool seg_path = !(s.flags & PIC_CONSERVE_FIX) && (gate || !(s.flags & PIC_MOMENTS));
    if (gate) {
        // decide the deferred cells from the last refreshed moments and draw
        // the judged sample; the queue then leaves deferred cells out of the
        // classes
        RC(launch_mom_select(c->gate_dev, step_dev, s.step, c->gate_mom_every, st));
        GateArgs g;
        memset(&g, 0, sizeof(g));
        g.moments = c->gate_mom;
        g.params = c->gate_params;
        g.M = n_cells;
        g.thr = c->gate_thr;
        g.kmax = c->gate_kmax;
        g.judge_thr = (uint64_t)floor(c->gate_judge_frac * 4294967296.0);
        g.bf16 = c->gate_bf16;
        g.seed = s.seed;
        g.step = s.step;
        g.step_dev = step_dev;
        g.k_acc = c->gate_k;
        g.skip = c->gate_skip;
        g.dt_scale = c->gate_dts;
        g.want = c->gate_want;
        g.prob = c->gate_prob;
        g.judge_list = c->gate_judge;
        g.g = c->gate_dev;
        g.analytic = c->gate_analytic;
        g.replicas = c->gate_replicas;
        g.dt = s.dt;
        g.lnL = s.lnL;
        g.tol = c->gate_tol;
        g.density = s.density;
        ktime_begin(KT_GATE, st);
        RC(launch_gate(g, st));
        ktime_end(KT_GATE, st);
    }
    ktime_begin(KT_QUEUE, st);
    RC(launch_build_queue(cs, n_cells, caps, lists, c->flags, gate ? c->gate_skip : nullptr,
                          mcc_thr != 0, seg_path ? &seg_scratch() : nullptr, seg_target(dtype), st));
    ktime_end(KT_QUEUE, st);

    if (gate) {
        RelaxArgs r;
        memset(&r, 0, sizeof(r));
        r.v = s.v;
        r.n = n;
        r.cell_start = cs;
        r.pid = s.pid;
        r.density = s.density;
        r.dt = s.dt;
        r.lnL = s.lnL;
        r.seed = s.seed;
        r.step = s.step;
        r.step_dev = step_dev;
        r.replicas = c->gate_replicas;
        r.list = c->gate_judge;
        r.count_dev = &c->gate_dev->judge_count;
        r.r_out = c->gate_r;
        r.dflags = c->flags;
        r.assume_sorted = assume ? 1 : 0;
        r.part = relax_part;
        r.cap = n_cells;
        ktime_begin(KT_RELAX, st);
        RC(launch_relax(dtype, r, c->num_cu, st));
        ktime_end(KT_RELAX, st);
        RC(launch_gate_score(c->gate_dev, c->gate_judge, c->gate_want, c->gate_r, c->gate_tol,
                             c->gate_max_false, c->gate_min_judged, st));
    }

    CollideArgs a;
    memset(&a, 0, sizeof(a));
    a.v = s.v;
    a.n = n;
    a.pid = s.pid;
    a.cell_start = cs;
    a.density = s.density;
    a.dt = s.dt;
    a.lnL = s.lnL;
    a.seed = s.seed;
    a.step = s.step;
    a.step_dev = step_dev;
    a.flags = s.flags;
    a.mcc_thr = mcc_thr;
    a.mass_ratio = c->mcc_mr;
    a.moments = c->moments_out;
    a.debt = (s.flags & PIC_CONSERVE_FIX) ? c->debt : nullptr;
    a.dflags = c->flags;
    a.order = order;
    if (gate) {
        // deferred cells are in no class queue: their null collisions run
        // here, and moment sums come from the pass after the collisions
        a.dt_scale = c->gate_dts;
        a.flags &= ~(uint32_t)PIC_MOMENTS;
        if (mcc_thr) {
            ktime_begin(KT_DEFER, st);
            RC(launch_deferred(dtype, a, lists, n_cells, c->num_cu, st));
            ktime_end(KT_DEFER, st);
        }
    }
    RC(launch_collide(dtype, a, lists, n_cells, caps, 0, c->num_cu, st, seg_path, s.live));
    if (s.flags & PIC_CHECK_FINITE) RC(launch_check_finite(dtype, s.v, n, c->flags, st));
    if (gate) {
        // the sums the next decision reads: post-step state, on refresh steps
        ktime_begin(KT_MOMENTS, st);
        RC(launch_moments(dtype, s.v, n, cs, n_cells, c->gate_mom, &c->gate_dev->mom_now, c->num_cu,
                          st));
        if ((s.flags & PIC_MOMENTS) && c->moments_out)
            RC(launch_moments(dtype, s.v, n, cs, n_cells, c->moments_out, nullptr, c->num_cu, st));
        ktime_end(KT_MOMENTS, st);
        RC(launch_gate_end(c->gate_dev, st));
    }
    return PIC_OK;
}

static int collide_common(pic_ctx *c, const StepArgs &s)
{
    RC(step_check(c, s));
    CK(hipSetDevice(c->device));
    RC(ensure_ws(c, step_ws_bytes(c, s)));
    if (s.flags & PIC_GATE) RC(ensure_gate(c, s.n_cells));
    if (s.flags & PIC_CONSERVE_FIX) RC(ensure_debt(c, s.n_cells));
    return step_enqueue(c, s, c->stream, nullptr);
}

int coulomb_collide(pic_ctx *c, int dtype, void *v, int32_t *cell_of, uint32_t *pid, int64_t n,
                    int32_t n_cells, double dt, double lnLambda, const double *density,
                    uint64_t seed, uint64_t step, uint32_t flags)
{
    if (!c) return PIC_ERR_ARG;
    const StepArgs s = {dtype, v, cell_of, pid, n, n_cells, dt, lnLambda, density, seed, step, flags};
    return collide_common(c, s);
}

int coulomb_collide_noalloc(pic_ctx *c, int dtype, void *v, int32_t *cell_of, uint32_t *pid,
                            int64_t n, int32_t n_cells, double dt, double lnLambda,
                            const double *density, uint64_t seed, uint64_t step, uint32_t flags)
{
    if (!c) return PIC_ERR_ARG;
    const StepArgs s = {dtype, v, cell_of, pid, n, n_cells, dt, lnLambda, density, seed, step,
                        flags | PIC_ASSUME_SORTED};
    if (flags & ~(uint32_t)(PIC_FUSE_MCC | PIC_ASSUME_SORTED | PIC_MOMENTS)) return PIC_ERR_ARG;
    RC(step_check(c, s));
    if (n_cells > PIC_NOALLOC_MAX_CELLS) return PIC_ERR_RANGE;
    const size_t cs_bytes = ((size_t)(n_cells + 1) * 4 + 255) & ~(size_t)255;
    static_assert(((size_t)(PIC_NOALLOC_MAX_CELLS + 1) * 4 + 255) / 256 * 256 +
                          (size_t)PIC_NOALLOC_MAX_CELLS * QUEUE_LISTS * 4 <=
                      PIC_NOALLOC_SCRATCH_BYTES,
                  "scratch holds the cell starts and work lists of the largest grid");
    if (!c->noalloc) return PIC_ERR_STATE;
    CK(hipSetDevice(c->device));
    hipStream_t st = c->stream;
    unsigned char *base = (unsigned char *)c->noalloc;
    int32_t *cs = (int32_t *)base;
    int32_t *lists = (int32_t *)(base + cs_bytes);
    // the default routing: every cell of the LDS classes, none beyond them
    const ClassCaps caps = collide_caps(dtype, c->lds_max);
    const uint64_t mcc_thr = (flags & PIC_FUSE_MCC) ? mcc_threshold(dt, c->mcc_sigma0, c->mcc_nn) : 0;
    RC(launch_reset_flags(c->flags, st));
    RC(launch_bin_check(cell_of, n, n_cells, cs, c->flags, 2, nullptr, st));
    RC(launch_build_queue(cs, n_cells, caps, lists, c->flags, nullptr, 0, nullptr, 0, st));
    RC(launch_reject_list(c->flags, caps.ncls, st));   // cells beyond the LDS classes
    CollideArgs a;
    memset(&a, 0, sizeof(a));
    a.v = v;
    a.n = n;
    a.pid = pid;
    a.cell_start = cs;
    a.density = density;
    a.dt = dt;
    a.lnL = lnLambda;
    a.seed = seed;
    a.step = step;
    a.flags = s.flags;
    a.mcc_thr = mcc_thr;
    a.mass_ratio = c->mcc_mr;
    a.moments = c->moments_out;
    a.dflags = c->flags;
    const uint32_t lds_classes = (1u << caps.ncls) - 1u;
    return launch_collide(dtype, a, lists, n_cells, caps, 0, c->num_cu, st, false, lds_classes);
}

int pic_run_steps(pic_ctx *c, int dtype, void *v, int32_t *cell_of, uint32_t *pid, int64_t n,
                  int32_t n_cells, double dt, double lnLambda, const double *density, uint64_t seed,
                  uint64_t step0, int64_t nsteps, uint32_t flags)
{
    if (!c || nsteps < 0) return PIC_ERR_ARG;
    if (nsteps == 0) return PIC_OK;
    StepArgs s = {dtype, v, cell_of, pid, n, n_cells, dt, lnLambda, density, seed, step0, flags};
    int64_t done = 0;
    if (!(flags & PIC_ASSUME_SORTED)) {
        RC(collide_common(c, s));          // first step: re-bins unsorted storage
        done = 1;
        if (nsteps == 1) return PIC_OK;
    } else {
        // every step is a replay: the same checks and scratch as an eager step
        RC(step_check(c, s));
        CK(hipSetDevice(c->device));
        RC(ensure_ws(c, step_ws_bytes(c, s)));
        if (s.flags & PIC_GATE) RC(ensure_gate(c, s.n_cells));
        if (s.flags & PIC_CONSERVE_FIX) RC(ensure_debt(c, s.n_cells));
    }
    // Later steps find the storage in cell order (the collision step never
    // changes cell membership): capture one such step once and replay it.
    // Nothing here waits for the device: size classes without cells are
    // launched and leave at once (their counts are read on the device).
    s.flags |= PIC_ASSUME_SORTED;
    s.step = 0;
    unsigned char key[sizeof(c->graph_key)];
    size_t kl = 0;
    bool key_full = false;
    auto put = [&](const void *p, size_t bytes) {
        if (kl + bytes > sizeof(key)) {
            key_full = true;
            return;
        }
        memcpy(key + kl, p, bytes);
        kl += bytes;
    };
    put(&s, sizeof(s));
    put(&c->ws, sizeof(c->ws));
    put(&c->mcc_sigma0, sizeof(double));
    put(&c->mcc_nn, sizeof(double));
    put(&c->mcc_mr, sizeof(double));
    put(&c->moments_out, sizeof(void *));
    put(&c->gate_params, sizeof(void *));
    put(&c->gate_thr, sizeof(float));
    put(&c->gate_kmax, sizeof(int));
    put(&c->gate_judge_frac, sizeof(double));
    put(&c->gate_mom_every, sizeof(int));
    put(&c->gate_tol, sizeof(double));
    put(&c->gate_replicas, sizeof(int));
    put(&c->gate_bf16, sizeof(int));
    put(&c->gate_analytic, sizeof(int));
    put(&c->gate_mem, sizeof(void *));
    put(&c->debt, sizeof(void *));
    put(&c->tuned_valid[dtype == PIC_F64], sizeof(bool));
    put(&c->tuned[dtype == PIC_F64], sizeof(ClassCaps));
    if (key_full) return PIC_ERR_STATE;   // the key outgrew its buffer: a build error, not a caller's
    if (!c->exec || kl != c->graph_key_len || memcmp(key, c->graph_key, kl) != 0) {
        if (c->exec) {
            CK(hipGraphExecDestroy(c->exec));
            c->exec = nullptr;
        }
        if (!c->cap_stream) CK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        const bool timing = ktime_pause();
        hipGraph_t g = nullptr;
        CK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        int rc = step_enqueue(c, s, c->cap_stream, c->step_dev);
        if (rc == PIC_OK) rc = launch_step_inc(c->step_dev, c->cap_stream);
        const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
        ktime_resume(timing);
        if (rc != PIC_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        CK(e);
        const hipError_t ei = hipGraphInstantiate(&c->exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        CK(ei);
        memcpy(c->graph_key, key, kl);
        c->graph_key_len = kl;
    }
    RC(launch_set_step(c->step_dev, step0 + (uint64_t)done, c->stream));
    for (int64_t k = done; k < nsteps; ++k) CK(hipGraphLaunch(c->exec, c->stream));
    return PIC_OK;
}

int mcc_null_collide(pic_ctx *c, int dtype, void *v, const uint32_t *pid, int64_t n, double dt,
                     double sigma0, double n_neutral, double mass_ratio, uint64_t seed,
                     uint64_t step, uint8_t *candidate_out)
{
    if (!c) return PIC_ERR_ARG;
    RC(check_dtype(dtype));
    if (n < 0 || !(dt > 0.0) || !(sigma0 >= 0.0) || !(n_neutral >= 0.0) || !(mass_ratio >= 0.0) ||
        !(mass_ratio < 0.5))
        return PIC_ERR_ARG;
    if (n > 0 && (!v || !pid)) return PIC_ERR_ARG;
    CK(hipSetDevice(c->device));
    ktime_begin(KT_MCC, c->stream);
    const int rc = launch_mcc(dtype, v, pid, n, mcc_threshold(dt, sigma0, n_neutral), mass_ratio,
                              seed, step, candidate_out, c->stream);
    ktime_end(KT_MCC, c->stream);
    return rc;
}

int mcc_null_collide_exact(pic_ctx *c, int dtype, void *v, const uint32_t *pid, int64_t n, double dt,
                           double sigma0, double n_neutral, double mass_ratio, uint64_t seed,
                           uint64_t step, uint8_t *selected_out)
{
    if (!c) return PIC_ERR_ARG;
    RC(check_dtype(dtype));
    if (n < 0 || !(dt > 0.0) || !(sigma0 >= 0.0) || !(n_neutral >= 0.0) || !(mass_ratio >= 0.0) ||
        !(mass_ratio < 0.5))
        return PIC_ERR_ARG;
    if (n > 0 && (!v || !pid)) return PIC_ERR_ARG;
    if (n > INT32_MAX) return PIC_ERR_ARG;   // slots and counts are 32-bit
    if (n == 0) return PIC_OK;
    CK(hipSetDevice(c->device));
    const double nu_max = n_neutral * sigma0 * sqrt(2.0);
    const double p = 1.0 - exp(-nu_max * dt);
    const int64_t k = (int64_t)llround(p * (double)n);
    RC(ensure_ws(c, mcc_exact_ws_bytes(n, k)));
    ktime_begin(KT_MCC, c->stream);
    const int rc = launch_mcc_exact(dtype, v, pid, n, k, mass_ratio, seed, step, selected_out, c->ws,
                                    c->stream);
    ktime_end(KT_MCC, c->stream);
    return rc;
}


// Nanbu's operator or the triplet variant on cell-ordered storage: the class
// kernels with that pair operator (cells beyond the LDS classes on one
// workgroup each).
static int variant_step(pic_ctx *c, int dtype, void *v, const uint32_t *pid, int64_t n,
                        const int32_t *cell_start, int32_t n_cells, double dt, double lnL,
                        const double *density, uint64_t seed, uint64_t step, int variant, int slot)
{
    if (!c || n < 0 || n > INT32_MAX || n_cells < 1 || !cell_start || !(dt > 0.0) || !(lnL > 0.0) ||
        (n > 0 && (!v || !pid)))
        return PIC_ERR_ARG;
    RC(check_dtype(dtype));
    if (n == 0) return PIC_OK;
    CK(hipSetDevice(c->device));
    hipStream_t st = c->stream;
    RC(ensure_ws(c, (size_t)n_cells * QUEUE_LISTS * 4 + huge_scratch_bytes(dtype, n) + 4096));
    Bump b(c->ws);
    int32_t *lists = (int32_t *)b.take((size_t)n_cells * QUEUE_LISTS * 4);
    set_huge_scratch(dtype, n, b.take(huge_scratch_bytes(dtype, n)));
    const ClassCaps caps = collide_caps(dtype, c->lds_max);
    ktime_begin(slot, st);
    RC(launch_reset_flags(c->flags, st));
    RC(launch_build_queue(cell_start, n_cells, caps, lists, c->flags, nullptr, 0, nullptr, 0, st));
    CollideArgs a;
    memset(&a, 0, sizeof(a));
    a.v = v;
    a.n = n;
    a.pid = pid;
    a.cell_start = cell_start;
    a.density = density;
    a.dt = dt;
    a.lnL = lnL;
    a.seed = seed;
    a.step = step;
    a.dflags = c->flags;
    a.variant = variant;
    const int rc = launch_collide(dtype, a, lists, n_cells, caps, 0, c->num_cu, st, false, ~0u);
    ktime_end(slot, st);
    return rc;
}

int coulomb_collide_nanbu(pic_ctx *c, int dtype, void *v, const uint32_t *pid, int64_t n,
                          const int32_t *cell_start, int32_t n_cells, double dt, double lnL,
                          const double *density, uint64_t seed, uint64_t step)
{
    return variant_step(c, dtype, v, pid, n, cell_start, n_cells, dt, lnL, density, seed, step,
                        VAR_NANBU, KT_NANBU);
}

int coulomb_collide_weighted(pic_ctx *c, int dtype, void *v, const void *w, const uint32_t *pid,
                             int64_t n, const int32_t *cell_start, int32_t n_cells, double dt,
                             double lnL, const double *density, uint64_t seed, uint64_t step,
                             uint32_t flags)
{
    if (!c || n < 0 || n > INT32_MAX || n_cells < 1 || !cell_start || !(dt > 0.0) || !(lnL > 0.0) ||
        (n > 0 && (!v || !w || !pid)))
        return PIC_ERR_ARG;
    RC(check_dtype(dtype));
    if (flags & ~(uint32_t)PIC_FUSE_MCC) return PIC_ERR_ARG;
    if ((flags & PIC_FUSE_MCC) && !c->mcc_set) return PIC_ERR_STATE;
    if (n == 0) return PIC_OK;
    CK(hipSetDevice(c->device));
    hipStream_t st = c->stream;
    RC(ensure_ws(c, (size_t)n_cells * QUEUE_LISTS * 4 + huge_scratch_bytes(dtype, n) + 4096));
    Bump b(c->ws);
    int32_t *lists = (int32_t *)b.take((size_t)n_cells * QUEUE_LISTS * 4);
    set_huge_scratch(dtype, n, b.take(huge_scratch_bytes(dtype, n)));
    const ClassCaps caps = collide_caps(dtype, c->lds_max);
    ktime_begin(KT_WEIGHTED, st);
    RC(launch_reset_flags(c->flags, st));
    RC(launch_build_queue(cell_start, n_cells, caps, lists, c->flags, nullptr, 0, nullptr, 0, st));
    CollideArgs a;
    memset(&a, 0, sizeof(a));
    a.v = v;
    a.w = w;
    a.n = n;
    a.pid = pid;
    a.cell_start = cell_start;
    a.density = density;
    a.dt = dt;
    a.lnL = lnL;
    a.seed = seed;
    a.step = step;
    a.mcc_thr = (flags & PIC_FUSE_MCC) ? mcc_threshold(dt, c->mcc_sigma0, c->mcc_nn) : 0;
    a.mass_ratio = c->mcc_mr;
    a.dflags = c->flags;
    const int rc = launch_collide(dtype, a, lists, n_cells, caps, 0, c->num_cu, st, false, ~0u);
    ktime_end(KT_WEIGHTED, st);
    return rc;
}

int coulomb_collide_triplet(pic_ctx *c, int dtype, void *v, const uint32_t *pid, int64_t n,
                            const int32_t *cell_start, int32_t n_cells, double dt, double lnL,
                            const double *density, uint64_t seed, uint64_t step)
{
    return variant_step(c, dtype, v, pid, n, cell_start, n_cells, dt, lnL, density, seed, step,
                        VAR_TRIPLET, KT_TRIPLET);
}

int recombine(pic_ctx *c, int dtype, void *v, void *w, const uint32_t *pid, const uint8_t *primary,
              int64_t n, const int32_t *cell_start, int32_t n_cells, double eps, uint64_t seed,
              uint64_t step, int32_t *events)
{
    if (!c || n < 0 || n > INT32_MAX || n_cells < 1 || !cell_start || !(eps >= 0.0) ||
        !(eps < 1e300) || (n > 0 && (!v || !w || !pid || !primary)))
        return PIC_ERR_ARG;
    RC(check_dtype(dtype));
    CK(hipSetDevice(c->device));
    RecombArgs a;
    a.v = v;
    a.w = w;
    a.pid = pid;
    a.primary = primary;
    a.n = n;
    a.cs = cell_start;
    a.M = n_cells;
    a.eps = eps;
    a.seed = seed;
    a.step = (uint32_t)step;
    a.events = events;
    ktime_begin(KT_RECOMB, c->stream);
    const int rc = launch_recombine(dtype, a, c->num_cu, c->stream);
    ktime_end(KT_RECOMB, c->stream);
    return rc;
}

int p2c_sums(pic_ctx *c, int dtype, const void *q, int32_t nq, const int32_t *cell_of, int64_t n,
             int32_t n_cells, double *out)
{
    if (!c || n < 0 || n_cells < 1 || nq < 1 || nq > 4 || !out || (n > 0 && (!q || !cell_of)))
        return PIC_ERR_ARG;
    if (n > INT32_MAX || (int64_t)n_cells * nq > (int64_t)1 << 28) return PIC_ERR_ARG;
    RC(check_dtype(dtype));
    CK(hipSetDevice(c->device));
    RC(ensure_ws(c, p2c_ws_bytes(n, n_cells, nq, c->num_cu)));
    ktime_begin(KT_P2C, c->stream);
    const int rc = launch_p2c(dtype, nq, q, cell_of, n, n_cells, out, c->ws, c->flags, c->num_cu, c->stream);
    ktime_end(KT_P2C, c->stream);
    return rc;
}

int pic_philox(pic_ctx *c, uint64_t seed, uint64_t step, uint32_t domain, uint32_t c3,
               const uint32_t *c0, int64_t n, uint32_t *out)
{
    if (!c || n < 0 || (n > 0 && (!c0 || !out))) return PIC_ERR_ARG;
    CK(hipSetDevice(c->device));
    return launch_philox(seed, step, domain, c3, c0, n, out, c->stream);
}

int coulomb_pairs(pic_ctx *c, const int32_t *cell_start, const uint32_t *pid, int32_t n_cells,
                  uint64_t seed, uint64_t step, int32_t *sorted, int32_t *partner)
{
    if (!c || !cell_start || n_cells < 1 || !sorted || !partner || !pid) return PIC_ERR_ARG;
    CK(hipSetDevice(c->device));
    int32_t nn = 0;
    CK(hipMemcpyAsync(&nn, cell_start + n_cells, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    CK(hipStreamSynchronize(c->stream));
    const int64_t n = nn;
    const size_t need = (size_t)n_cells * QUEUE_LISTS * 4 + huge_scratch_bytes(PIC_F32, n) + 4096;
    RC(ensure_ws(c, need));
    Bump b(c->ws);
    int32_t *lists = (int32_t *)b.take((size_t)n_cells * QUEUE_LISTS * 4);
    set_huge_scratch(PIC_F32, n, b.take(huge_scratch_bytes(PIC_F32, n)));
    RC(launch_reset_flags(c->flags, c->stream));
    const ClassCaps caps = collide_caps(PIC_F32, c->lds_max);
    RC(launch_build_queue(cell_start, n_cells, caps, lists, c->flags, nullptr, 0, nullptr, 0,
                          c->stream));
    CollideArgs a;
    memset(&a, 0, sizeof(a));
    a.n = n;
    a.pid = pid;
    a.cell_start = cell_start;
    a.dt = 1.0;
    a.lnL = 1.0;
    a.seed = seed;
    a.step = step;
    a.dflags = c->flags;
    a.sorted_out = sorted;
    a.partner_out = partner;
    return launch_collide(PIC_F32, a, lists, n_cells, caps, 1, c->num_cu, c->stream);
}

int pic_cell_moments(pic_ctx *c, int dtype, const void *v, int64_t n, const int32_t *cell_start,
                     int32_t n_cells, double *out)
{
    if (!c || n < 0 || n_cells < 1 || !cell_start || !out || (n > 0 && !v)) return PIC_ERR_ARG;
    RC(check_dtype(dtype));
    CK(hipSetDevice(c->device));
    return launch_moments(dtype, v, n, cell_start, n_cells, out, nullptr, c->num_cu, c->stream);
}

int pic_unsort(pic_ctx *c, int dtype, void *v, uint32_t *pid, int32_t *cell_of, int64_t n)
{
    if (!c || n < 0 || (n > 0 && (!v || !pid || !cell_of))) return PIC_ERR_ARG;
    RC(check_dtype(dtype));
    CK(hipSetDevice(c->device));
    const size_t es = dtype == PIC_F32 ? 4 : 8;
    RC(ensure_ws(c, (size_t)n * (3 * es + 4) + 1024));
    return launch_unsort(dtype, v, pid, cell_of, n, c->ws, c->stream);
}

static std::vector<ClassCaps> tune_candidates(const ClassCaps &b)
{
    std::vector<ClassCaps> v;
    auto add = [&](ClassCaps c) { v.push_back(c); };
    add(b);                                   // one launch per size class
    ClassCaps c = b;
    c.cap[0] = b.cap[0] / 2;                  // fewer cells on the 256-thread class
    add(c);
    c = b;
    c.cap[2] = b.cap[1];                      // 2049..4096-member cells on the largest class
    add(c);
    c = b;
    c.cap[1] = b.cap[0];                      // 513..2048-member cells on the 1024-thread classes
    add(c);
    c = b;
    c.blocks_per_cu[3] = 2;                   // two resident workgroups per CU on the largest class
    add(c);
    c = b;
    c.blocks_per_cu[0] = 16;
    c.blocks_per_cu[1] = 8;
    add(c);
    c = b;
    c.blocks_per_cu[4] = 2;
    add(c);
    ClassCaps u = b;
    u.unified = 1;                            // one persistent launch, small cells one wave each
    u.wave = 1;
    add(u);
    c = u;
    c.wave = 0;                               // ... every cell on a whole workgroup
    add(c);
    c = u;
    c.cap[0] = b.cap[0] / 2;                  // ... fewer cells on the wave schedule
    add(c);
    return v;
}

int pic_set_workspace_limit(pic_ctx *c, size_t bytes)
{
    if (!c) return PIC_ERR_ARG;
    c->ws_limit = bytes;
    return PIC_OK;
}

int pic_set_schedule(pic_ctx *c, int dtype, int schedule)
{
    if (!c || schedule < 0 || schedule > 2) return PIC_ERR_ARG;
    RC(check_dtype(dtype));
    const int di = dtype == PIC_F64;
    ClassCaps caps = c->tuned_valid[di] ? c->tuned[di] : collide_caps(dtype, c->lds_max);
    caps.unified = schedule != 0;
    caps.wave = schedule == 1;
    c->tuned[di] = caps;
    c->tuned_valid[di] = true;
    return PIC_OK;
}

int pic_autotune(pic_ctx *c, int dtype, const void *v, const int32_t *cell_of, const uint32_t *pid,
                 int64_t n, int32_t n_cells, double dt, double lnLambda, uint32_t flags,
                 int32_t *choice_out)
{
    if (!c) return PIC_ERR_ARG;
    flags &= ~(uint32_t)(PIC_GATE | PIC_MOMENTS | PIC_ASSUME_SORTED);
    StepArgs s = {dtype, nullptr, nullptr, nullptr, n, n_cells, dt, lnLambda, nullptr, 0, 0, flags};
    s.v = (void *)v;
    s.cell_of = (int32_t *)cell_of;
    s.pid = (uint32_t *)pid;
    RC(step_check(c, s));
    CK(hipSetDevice(c->device));
    const size_t es = dtype == PIC_F32 ? 4 : 8;
    const int di = dtype == PIC_F64;
    // a scratch copy of the state: the caller's arrays are not modified
    void *copy = nullptr;
    const size_t vb = (size_t)n * 3 * es, ib = (size_t)n * 4;
    const size_t db = (size_t)n_cells * 4 * sizeof(double);
    if (hipMalloc(&copy, vb + 2 * ib + db + 1024) != hipSuccess) {
        (void)hipGetLastError();
        return PIC_ERR_NOMEM;
    }
    Bump b(copy);
    StepArgs t = s;
    t.v = b.take(vb);
    t.cell_of = (int32_t *)b.take(ib);
    t.pid = (uint32_t *)b.take(ib);
    // trial steps carry their conservation shortfall in a scratch buffer, so
    // the context's per-cell state is left as it was
    double *const saved_debt = c->debt;
    const int32_t saved_debt_M = c->debt_M;
    c->debt = (double *)b.take(db);
    c->debt_M = n_cells;
    int rc = hipMemsetAsync(c->debt, 0, db, c->stream) == hipSuccess ? PIC_OK : PIC_ERR_HIP;
    std::vector<int32_t> hcs((size_t)n_cells + 1);
    std::string key;
    const ClassCaps base = collide_caps(dtype, c->lds_max);
    const std::vector<ClassCaps> cands = tune_candidates(base);
    int best = 0;
    float best_ms = 1e30f;
    bool cached = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    do {
        if (rc != PIC_OK) break;
        if (hipMemcpyAsync(t.v, v, vb, hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
            hipMemcpyAsync(t.cell_of, cell_of, ib, hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
            hipMemcpyAsync(t.pid, pid, ib, hipMemcpyDeviceToDevice, c->stream) != hipSuccess) {
            rc = PIC_ERR_HIP;
            break;
        }
        c->tuned_valid[di] = false;
        if ((rc = collide_common(c, t)) != PIC_OK) break;     // re-bins the copy
        // the histogram of log2 cell sizes keys the cache
        int32_t *cs = (int32_t *)c->ws;
        if (hipMemcpyAsync(hcs.data(), cs, hcs.size() * 4, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess) {
            rc = PIC_ERR_HIP;
            break;
        }
        long long hist[34] = {0};
        for (int32_t j = 0; j < n_cells; ++j) {
            const int64_t cnt = hcs[j + 1] - hcs[j];
            int bkt = 0;
            while (bkt < 33 && ((int64_t)1 << bkt) < cnt) ++bkt;
            hist[bkt] += 1;
        }
        hipDeviceProp_t prop;
        const char *arch = hipGetDeviceProperties(&prop, c->device) == hipSuccess ? prop.gcnArchName : "?";
        char buf[512];
        snprintf(buf, sizeof(buf), "%s|%d|%lld|%d|%u|", arch, dtype, (long long)n, n_cells, flags);
        key = buf;
        for (int k = 0; k < 34; ++k)
            if (hist[k]) {
                snprintf(buf, sizeof(buf), "%d:%lld,", k, hist[k]);
                key += buf;
            }
        const char *path = getenv("PICCOLL_TUNE_CACHE");
        if (path) {
            FILE *f = fopen(path, "r");
            if (f) {
                char line[2048];
                while (fgets(line, sizeof(line), f)) {
                    // line: {"key": "<key>", "choice": <k>, "ms": <t>}
                    const std::string ln(line);
                    const std::string pre = "{\"key\": \"" + key + "\", \"choice\": ";
                    if (ln.compare(0, pre.size(), pre) == 0) {
                        const int ch = atoi(ln.c_str() + pre.size());
                        if (ch >= 0 && ch < (int)cands.size()) {
                            best = ch;
                            cached = true;
                        }
                    }
                }
                fclose(f);
            }
        }
        if (cached) break;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            rc = PIC_ERR_HIP;
            break;
        }
        t.flags |= PIC_ASSUME_SORTED;
        for (size_t k = 0; k < cands.size() && rc == PIC_OK; ++k) {
            c->tuned[di] = cands[k];
            c->tuned_valid[di] = true;
            if ((rc = collide_common(c, t)) != PIC_OK) break;   // warm-up
            (void)hipEventRecord(e0, c->stream);
            for (int r = 0; r < 3 && rc == PIC_OK; ++r) {
                t.step = 1 + r;
                rc = collide_common(c, t);
            }
            (void)hipEventRecord(e1, c->stream);
            float ms = 0.0f;
            if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = PIC_ERR_HIP;
                break;
            }
            if (ms < best_ms) {
                best_ms = ms;
                best = (int)k;
            }
        }
        if (rc == PIC_OK && path) {
            FILE *f = fopen(path, "a");
            if (f) {
                fprintf(f, "{\"key\": \"%s\", \"choice\": %d, \"ms\": %.5f}\n", key.c_str(), best,
                        best_ms / 3.0f);
                fclose(f);
            }
        }
    } while (0);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(c->stream);
    c->debt = saved_debt;
    c->debt_M = saved_debt_M;
    (void)hipFree(copy);
    if (rc != PIC_OK) {
        c->tuned_valid[di] = false;
        return rc;
    }
    c->tuned[di] = cands[best];
    c->tuned_valid[di] = true;
    if (choice_out) *choice_out = best;
    return PIC_OK;
}

}  // extern "C"

// pic_api.cpp -- the C ABI: context, argument checks, scratch management and
// the order of launches of one collision step.
#include <math.h>
#include <string.h>

#include <new>
#include <vector>

#include "pic_internal.hpp"

struct pic_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cu = 256;
    size_t lds_max = 65536;
    DevFlags *flags = nullptr;
    void *ws = nullptr;
    size_t ws_cap = 0;
    double mcc_sigma0 = 0.0, mcc_nn = 0.0, mcc_mr = 0.0;
    bool mcc_set = false;
    double *moments_out = nullptr;
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
    CK(hipSetDevice(c->device));
    CK(hipStreamSynchronize(c->stream));
    if (c->ws) {
        CK(hipFree(c->ws));
        c->ws = nullptr;
        c->ws_cap = 0;
    }
    const size_t want = bytes + bytes / 8;
    if (hipMalloc(&c->ws, want) != hipSuccess) {
        (void)hipGetLastError();
        c->ws = nullptr;
        return PIC_ERR_NOMEM;
    }
    c->ws_cap = want;
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

int sort_by_cell(pic_ctx *c, const SortStreams &caller, const SortStreams &tmp, int64_t n,
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
        RC(radix_pass(p, bs, c->stream));
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
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && v > 0)
        c->num_cu = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && v > 0)
        c->lds_max = (size_t)v;
    if (hipMalloc((void **)&c->flags, sizeof(DevFlags)) != hipSuccess) {
        delete c;
        return PIC_ERR_NOMEM;
    }
    if (hipMemset(c->flags, 0, sizeof(DevFlags)) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(c->flags);
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
    if (c->ws) (void)hipFree(c->ws);
    if (c->flags) (void)hipFree(c->flags);
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
    int host[4] = {0, 0, 0, 0};
    CK(hipMemcpy(host, c->flags, sizeof(host), hipMemcpyDeviceToHost));
    if (host[2] || host[3]) {
        const int zero[2] = {0, 0};
        CK(hipMemcpy(&c->flags->sticky_range, zero, sizeof(zero), hipMemcpyHostToDevice));
    }
    if (host[2]) return PIC_ERR_RANGE;
    if (host[3]) return PIC_ERR_STATE;
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

static int collide_common(pic_ctx *c, int dtype, void *v, int32_t *cell_of, uint32_t *pid, int64_t n,
                          int32_t n_cells, double dt, double lnL, const double *density,
                          uint64_t seed, uint64_t step, uint32_t flags)
{
    RC(check_dtype(dtype));
    if (n < 0 || n > INT32_MAX || n_cells < 1 || n_cells > (1 << 24) || !(dt > 0.0) || !(lnL > 0.0))
        return PIC_ERR_ARG;
    if (n > 0 && (!v || !cell_of || !pid)) return PIC_ERR_ARG;
    if ((flags & PIC_FUSE_MCC) && !c->mcc_set) return PIC_ERR_STATE;
    if ((flags & PIC_MOMENTS) && !c->moments_out) return PIC_ERR_STATE;
    CK(hipSetDevice(c->device));
    const size_t es = dtype == PIC_F32 ? 4 : 8;
    const size_t need = (size_t)(n_cells + 1) * 4 + (size_t)n_cells * 5 * 4 + (size_t)n * (8 + 3 * es) +
                        radix_scratch_bytes(n) + huge_scratch_bytes(dtype, n) + 8192;
    RC(ensure_ws(c, need));
    Bump b(c->ws);
    int32_t *cs = (int32_t *)b.take((size_t)(n_cells + 1) * 4);
    int32_t *lists = (int32_t *)b.take((size_t)n_cells * 5 * 4);
    int32_t *tkey = (int32_t *)b.take((size_t)n * 4);
    uint32_t *tpid = (uint32_t *)b.take((size_t)n * 4);
    void *tv = b.take((size_t)n * 3 * es);
    BinScratch bs;
    bs.hist = (uint32_t *)b.take(radix_scratch_bytes(n));
    bs.bsum = bs.hist + 256 * ((n + 4095) / 4096 + 1);
    set_huge_scratch(dtype, n, b.take(huge_scratch_bytes(dtype, n)));

    RC(launch_reset_flags(c->flags, c->stream));
    const bool assume = (flags & PIC_ASSUME_SORTED) != 0;
    ktime_begin(KT_CHECK, c->stream);
    RC(launch_bin_check(cell_of, n, n_cells, cs, c->flags, assume ? 2 : 1, nullptr, c->stream));
    ktime_end(KT_CHECK, c->stream);
    if (!assume && n > 1 && n_cells > 1) {
        ktime_begin(KT_SORT, c->stream);
        SortStreams caller, tmp;
        memset(&caller, 0, sizeof(caller));
        memset(&tmp, 0, sizeof(tmp));
        caller.key = cell_of;
        tmp.key = tkey;
        caller.n32 = tmp.n32 = 1;
        caller.p32[0] = pid;
        tmp.p32[0] = tpid;
        if (dtype == PIC_F32) {
            caller.n32 = tmp.n32 = 4;
            for (int k = 0; k < 3; ++k) {
                caller.p32[1 + k] = (uint32_t *)v + (size_t)k * n;
                tmp.p32[1 + k] = (uint32_t *)tv + (size_t)k * n;
            }
        } else {
            caller.n64 = tmp.n64 = 3;
            for (int k = 0; k < 3; ++k) {
                caller.p64[k] = (uint64_t *)v + (size_t)k * n;
                tmp.p64[k] = (uint64_t *)tv + (size_t)k * n;
            }
        }
        RC(sort_by_cell(c, caller, tmp, n, n_cells, bs, &c->flags->unsorted));
        RC(launch_bin_check(cell_of, n, n_cells, cs, c->flags, 0, &c->flags->unsorted, c->stream));
        ktime_end(KT_SORT, c->stream);
    }
    const ClassCaps caps = collide_caps(dtype, c->lds_max);
    ktime_begin(KT_QUEUE, c->stream);
    RC(launch_build_queue(cs, n_cells, caps, lists, c->flags, c->stream));
    ktime_end(KT_QUEUE, c->stream);

    CollideArgs a;
    memset(&a, 0, sizeof(a));
    a.v = v;
    a.n = n;
    a.pid = pid;
    a.cell_start = cs;
    a.density = density;
    a.dt = dt;
    a.lnL = lnL;
    a.seed = seed;
    a.step = step;
    a.flags = flags;
    a.mcc_thr = (flags & PIC_FUSE_MCC) ? mcc_threshold(dt, c->mcc_sigma0, c->mcc_nn) : 0;
    a.mass_ratio = c->mcc_mr;
    a.moments = c->moments_out;
    a.dflags = c->flags;
    return launch_collide(dtype, a, lists, n_cells, caps, 0, c->num_cu, c->stream);
}

int coulomb_collide(pic_ctx *c, int dtype, void *v, int32_t *cell_of, uint32_t *pid, int64_t n,
                    int32_t n_cells, double dt, double lnLambda, const double *density,
                    uint64_t seed, uint64_t step, uint32_t flags)
{
    if (!c) return PIC_ERR_ARG;
    return collide_common(c, dtype, v, cell_of, pid, n, n_cells, dt, lnLambda, density, seed, step,
                          flags);
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
    const size_t need = (size_t)n_cells * 5 * 4 + huge_scratch_bytes(PIC_F32, n) + 4096;
    RC(ensure_ws(c, need));
    Bump b(c->ws);
    int32_t *lists = (int32_t *)b.take((size_t)n_cells * 5 * 4);
    set_huge_scratch(PIC_F32, n, b.take(huge_scratch_bytes(PIC_F32, n)));
    RC(launch_reset_flags(c->flags, c->stream));
    const ClassCaps caps = collide_caps(PIC_F32, c->lds_max);
    RC(launch_build_queue(cell_start, n_cells, caps, lists, c->flags, c->stream));
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
    return launch_moments(dtype, v, n, cell_start, n_cells, out, c->stream);
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

}  // extern "C"

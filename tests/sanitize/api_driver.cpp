// The library's host code under the address and undefined-behaviour
// sanitizers (host instrumentation only; device code is built as usual).
//   api_driver_asan            argument checks that need no device: every
//                              status string, every entry point with a NULL
//                              context or out-of-range arguments
//   api_driver_asan --device   the same, then a short session on device 0:
//                              re-binning, both dtypes, fused null
//                              collisions, conservation, replayed steps, the
//                              allocation-free form, the variants on cell
//                              starts, a workspace cap, an injected NaN,
//                              kernel timing, and the teardown
// Prints "api driver ok" and exits 0 when every call returned what it should.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include <hip/hip_runtime_api.h>

#include "piccoll.h"

#define EXPECT(x, want)                                                         \
    do {                                                                        \
        const int rc_ = (x);                                                    \
        if (rc_ != (want)) {                                                    \
            fprintf(stderr, "line %d: %s returned %d, want %d\n", __LINE__, #x, \
                    rc_, (int)(want));                                          \
            return 1;                                                           \
        }                                                                       \
    } while (0)

#define HIP_OK(x)                                                    \
    do {                                                             \
        if ((x) != hipSuccess) {                                     \
            fprintf(stderr, "line %d: %s failed\n", __LINE__, #x);   \
            return 1;                                                \
        }                                                            \
    } while (0)

static int no_device_checks()
{
    for (int s = 0; s <= 8; ++s)
        if (!pic_strerror(s) || !strlen(pic_strerror(s))) return 1;
    pic_ctx *c = nullptr;
    EXPECT(pic_create(nullptr, 0, nullptr), PIC_ERR_ARG);
    EXPECT(pic_create(&c, -1, nullptr), PIC_ERR_ARG);
    if (c) return 1;
    pic_destroy(nullptr);
    float v[3] = {0, 0, 0};
    int32_t cell = 0, cs[2] = {0, 1}, order = 0;
    uint32_t pid = 0;
    EXPECT(pic_sync(nullptr), PIC_ERR_ARG);
    EXPECT(pic_bin_cells(nullptr, &cell, 1, 1, cs, &order), PIC_ERR_ARG);
    EXPECT(coulomb_collide(nullptr, PIC_F32, v, &cell, &pid, 1, 1, 0.01, 10.0, nullptr, 0, 0, 0),
           PIC_ERR_ARG);
    EXPECT(coulomb_collide_noalloc(nullptr, PIC_F32, v, &cell, &pid, 1, 1, 0.01, 10.0, nullptr, 0,
                                   0, 0),
           PIC_ERR_ARG);
    EXPECT(pic_run_steps(nullptr, PIC_F32, v, &cell, &pid, 1, 1, 0.01, 10.0, nullptr, 0, 0, 2, 0),
           PIC_ERR_ARG);
    EXPECT(mcc_null_collide(nullptr, PIC_F32, v, &pid, 1, 0.01, 1.0, 1.0, 0.0, 0, 0, nullptr),
           PIC_ERR_ARG);
    EXPECT(coulomb_collide_weighted(nullptr, PIC_F32, v, v, &pid, 1, cs, 1, 0.01, 10.0, nullptr, 0,
                                    0, 0),
           PIC_ERR_ARG);
    EXPECT(coulomb_collide_nanbu(nullptr, PIC_F32, v, &pid, 1, cs, 1, 0.01, 10.0, nullptr, 0, 0),
           PIC_ERR_ARG);
    EXPECT(coulomb_collide_triplet(nullptr, PIC_F32, v, &pid, 1, cs, 1, 0.01, 10.0, nullptr, 0, 0),
           PIC_ERR_ARG);
    EXPECT(pic_set_schedule(nullptr, PIC_F32, 1), PIC_ERR_ARG);
    EXPECT(pic_set_workspace_limit(nullptr, 1), PIC_ERR_ARG);
    EXPECT(pic_set_mcc(nullptr, 1.0, 1.0, 0.0), PIC_ERR_ARG);
    EXPECT(pic_time_kernels(nullptr, 1), PIC_ERR_ARG);
    return 0;
}

// xorshift64* stream and Box-Muller normals for the host-side inputs
static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static double uni()
{
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return ((rng_state * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0) + 1e-300;
}
static double normal() { return sqrt(-2.0 * log(uni())) * cos(6.283185307179586 * uni()); }

static int device_session()
{
    const int32_t sizes[] = {0, 1, 3, 700, 1500, 2, 4097};
    const int32_t ncell = (int32_t)(sizeof(sizes) / sizeof(sizes[0]));
    std::vector<int32_t> cell;
    for (int32_t j = 0; j < ncell; ++j)
        for (int32_t k = 0; k < sizes[j]; ++k) cell.push_back(j);
    const int64_t n = (int64_t)cell.size();
    for (int64_t i = n - 1; i > 0; --i) {  // shuffled storage: the first step re-bins
        const int64_t r = (int64_t)(uni() * (double)(i + 1)) % (i + 1);
        const int32_t t = cell[i];
        cell[i] = cell[r];
        cell[r] = t;
    }
    std::vector<float> v32(3 * n);
    std::vector<double> v64(3 * n);
    std::vector<uint32_t> pid(n);
    for (int64_t i = 0; i < n; ++i) {
        pid[i] = (uint32_t)i;
        for (int d = 0; d < 3; ++d) v64[3 * i + d] = normal(), v32[3 * i + d] = (float)v64[3 * i + d];
    }

    pic_ctx *c = nullptr;
    EXPECT(pic_create(&c, 0, nullptr), PIC_OK);
    float *dv32, *dw;
    double *dv64;
    int32_t *dcell, *dcell64, *dcs, *dorder;
    uint32_t *dpid, *dpid64;
    HIP_OK(hipMalloc((void **)&dv32, 12 * n));
    HIP_OK(hipMalloc((void **)&dv64, 24 * n));
    HIP_OK(hipMalloc((void **)&dw, 4 * n));
    HIP_OK(hipMalloc((void **)&dcell, 4 * n));
    HIP_OK(hipMalloc((void **)&dcell64, 4 * n));
    HIP_OK(hipMalloc((void **)&dpid, 4 * n));
    HIP_OK(hipMalloc((void **)&dpid64, 4 * n));
    HIP_OK(hipMalloc((void **)&dcs, 4 * (ncell + 1)));
    HIP_OK(hipMalloc((void **)&dorder, 4 * n));
    HIP_OK(hipMemcpy(dv32, v32.data(), 12 * n, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(dv64, v64.data(), 24 * n, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(dcell, cell.data(), 4 * n, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(dcell64, cell.data(), 4 * n, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(dpid, pid.data(), 4 * n, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(dpid64, pid.data(), 4 * n, hipMemcpyHostToDevice));
    std::vector<float> ones(n, 1.0f);
    HIP_OK(hipMemcpy(dw, ones.data(), 4 * n, hipMemcpyHostToDevice));

    const double dt = 0.05, lnl = 10.0;
    // a workspace cap too small for the re-binning step: refused, nothing runs
    EXPECT(pic_set_workspace_limit(c, 64), PIC_OK);
    EXPECT(coulomb_collide(c, PIC_F32, dv32, dcell, dpid, n, ncell, dt, lnl, nullptr, 1, 0, 0),
           PIC_ERR_NOMEM);
    EXPECT(pic_set_workspace_limit(c, 0), PIC_OK);
    EXPECT(coulomb_collide(c, PIC_F32, dv32, dcell, dpid, n, ncell, dt, lnl, nullptr, 1, 0, 0),
           PIC_OK);
    EXPECT(pic_sync(c), PIC_OK);
    EXPECT(pic_set_mcc(c, 0.5, 1.0, 0.0), PIC_OK);
    EXPECT(pic_time_kernels(c, 1), PIC_OK);
    EXPECT(coulomb_collide(c, PIC_F32, dv32, dcell, dpid, n, ncell, dt, lnl, nullptr, 1, 1,
                           PIC_FUSE_MCC | PIC_ASSUME_SORTED | PIC_CHECK_FINITE),
           PIC_OK);
    EXPECT(pic_run_steps(c, PIC_F32, dv32, dcell, dpid, n, ncell, dt, lnl, nullptr, 1, 2, 4,
                         PIC_FUSE_MCC | PIC_ASSUME_SORTED),
           PIC_OK);
    EXPECT(pic_sync(c), PIC_OK);
    double ms[20];
    int64_t cnt[20];
    EXPECT(pic_kernel_times(c, ms, cnt), PIC_OK);
    EXPECT(pic_time_kernels(c, 0), PIC_OK);
    EXPECT(pic_set_schedule(c, PIC_F32, 1), PIC_OK);
    EXPECT(coulomb_collide(c, PIC_F32, dv32, dcell, dpid, n, ncell, dt, lnl, nullptr, 1, 6,
                           PIC_ASSUME_SORTED),
           PIC_OK);
    EXPECT(pic_set_schedule(c, PIC_F32, 0), PIC_OK);
    EXPECT(coulomb_collide_noalloc(c, PIC_F32, dv32, dcell, dpid, n, ncell, dt, lnl, nullptr, 1, 7,
                                   PIC_ASSUME_SORTED),
           PIC_OK);
    EXPECT(pic_sync(c), PIC_OK);

    // binary64 with the conservation fix, re-binning its own copy
    EXPECT(coulomb_collide(c, PIC_F64, dv64, dcell64, dpid64, n, ncell, dt, lnl, nullptr, 2, 0,
                           PIC_CONSERVE_FIX),
           PIC_OK);
    EXPECT(coulomb_collide(c, PIC_F64, dv64, dcell64, dpid64, n, ncell, dt, lnl, nullptr, 2, 1,
                           PIC_CONSERVE_FIX | PIC_ASSUME_SORTED),
           PIC_OK);
    EXPECT(pic_conserve_reset(c), PIC_OK);
    EXPECT(pic_sync(c), PIC_OK);

    // the variants on cell starts of the sorted binary32 storage
    EXPECT(pic_bin_cells(c, dcell, n, ncell, dcs, dorder), PIC_OK);
    EXPECT(coulomb_collide_nanbu(c, PIC_F32, dv32, dpid, n, dcs, ncell, dt, lnl, nullptr, 3, 0),
           PIC_OK);
    EXPECT(coulomb_collide_triplet(c, PIC_F32, dv32, dpid, n, dcs, ncell, dt, lnl, nullptr, 3, 1),
           PIC_OK);
    EXPECT(coulomb_collide_weighted(c, PIC_F32, dv32, dw, dpid, n, dcs, ncell, dt, lnl, nullptr, 3,
                                    2, PIC_FUSE_MCC),
           PIC_OK);
    EXPECT(mcc_null_collide(c, PIC_F32, dv32, dpid, n, dt, 0.5, 1.0, 0.0, 3, 3, nullptr), PIC_OK);
    EXPECT(pic_sync(c), PIC_OK);

    // one NaN: the finite check reports it once
    const float nan = NAN;
    HIP_OK(hipMemcpy(dv32 + 3 * 5, &nan, 4, hipMemcpyHostToDevice));
    EXPECT(coulomb_collide(c, PIC_F32, dv32, dcell, dpid, n, ncell, dt, lnl, nullptr, 4, 0,
                           PIC_ASSUME_SORTED | PIC_CHECK_FINITE),
           PIC_OK);
    EXPECT(pic_sync(c), PIC_ERR_NONFINITE);
    EXPECT(pic_sync(c), PIC_OK);

    pic_destroy(c);
    HIP_OK(hipFree(dv32));
    HIP_OK(hipFree(dv64));
    HIP_OK(hipFree(dw));
    HIP_OK(hipFree(dcell));
    HIP_OK(hipFree(dcell64));
    HIP_OK(hipFree(dpid));
    HIP_OK(hipFree(dpid64));
    HIP_OK(hipFree(dcs));
    HIP_OK(hipFree(dorder));
    return 0;
}

int main(int argc, char **argv)
{
    if (no_device_checks()) return 1;
    if (argc > 1 && !strcmp(argv[1], "--device") && device_session()) return 1;
    puts("api driver ok");
    return 0;
}

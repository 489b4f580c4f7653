// pic_misc.hip -- stand-alone null-collision step, per-cell moment sums,
// Philox export and the pid-order restore.
#include "pic_internal.hpp"

#define HIP_OK(x) do { if ((x) != hipSuccess) return PIC_ERR_HIP; } while (0)

namespace {

// One particle per lane: the candidate test needs only pid (4 B); velocities
// are read and written for candidates only (P_null of the particles).
template <typename R>
__global__ __launch_bounds__(256) void k_mcc(R *__restrict__ v, const uint32_t *__restrict__ pid,
                                             int64_t n, uint64_t thr, double mass_ratio,
                                             uint64_t seed, uint32_t step,
                                             uint8_t *__restrict__ cand_out)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t p = pid[i];
        const W4 w = draw4(seed, p, step, 0u, 0u);
        const bool c = (uint64_t)w.y < thr;
        if (cand_out) cand_out[i] = (uint8_t)c;
        if (c) {
            R x = v[i], y = v[n + i], z = v[2 * n + i];
            const W4 m = draw4(seed, p, step, 1u, 0u);
            scatter_dir(x, y, z, m, mass_ratio);
            v[i] = x;
            v[n + i] = y;
            v[2 * n + i] = z;
        }
    }
}

__global__ void k_philox(uint64_t seed, uint32_t step, uint32_t domain, uint32_t c3,
                         const uint32_t *__restrict__ c0, int64_t n, uint4 *__restrict__ out)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const W4 w = draw4(seed, c0[i], step, domain, c3);
        out[i] = make_uint4(w.x, w.y, w.z, w.w);
    }
}

// Per-cell moment sums, streamed.  A workgroup takes groups of four
// consecutive cells (round-robin, no atomics): first each wave sums one cell
// of at most MOM_WAVE_MAX members on its own (four members' loads in flight
// per lane, a wave reduce-scatter, no barriers), then the whole workgroup
// sums each larger cell of the group.
constexpr int MOM_T = 256;
constexpr int MOM_WAVE_MAX = 4096;

__device__ __forceinline__ void mom_add(double (&m)[16], double x, double y, double z)
{
    const double q2 = x * x + y * y + z * z;
    m[1] += x; m[2] += y; m[3] += z;
    m[4] += x * x; m[5] += y * y; m[6] += z * z;
    m[7] += x * y; m[8] += x * z; m[9] += y * z;
    m[10] += q2 * x; m[11] += q2 * y; m[12] += q2 * z;
    m[13] += q2 * q2;
}

// Sums members [i, hi) with stride `stride` into m (m[0] is left alone).
template <typename R>
__device__ __forceinline__ void mom_range(double (&m)[16], const R *__restrict__ v, int64_t n,
                                          int64_t i, int64_t hi, int stride)
{
    for (; i < hi; i += 4 * (int64_t)stride) {
        R x[4], y[4], z[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t e = i + (int64_t)k * stride;
            x[k] = y[k] = z[k] = (R)0;
            if (e < hi) {
                x[k] = v[e];
                y[k] = v[n + e];
                z[k] = v[2 * n + e];
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (i + (int64_t)k * stride < hi) mom_add(m, x[k], y[k], z[k]);
    }
}

template <typename R>
__global__ __launch_bounds__(MOM_T) void k_moments(const R *__restrict__ v, int64_t n,
                                                   const int32_t *__restrict__ cs, int32_t n_cells,
                                                   double *__restrict__ out, const int *run_if)
{
    __shared__ double red[16 * (MOM_T / PIC_WAVE)];
    if (run_if && !*run_if) return;
    const int lane = threadIdx.x & (PIC_WAVE - 1), wid = threadIdx.x / PIC_WAVE;
    constexpr int CPG = MOM_T / PIC_WAVE;    // cells per group
    const int groups = (n_cells + CPG - 1) / CPG;
    for (int g = blockIdx.x; g < groups; g += gridDim.x) {
        const int j = g * CPG + wid;
        if (j < n_cells) {
            const int lo = cs[j], cnt = cs[j + 1] - lo;
            if (cnt <= MOM_WAVE_MAX) {
                double m[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) m[q] = 0.0;
                mom_range<R>(m, v, n, lo + lane, (int64_t)lo + cnt, PIC_WAVE);
                // lane L holds sum L / 4 of the wave
                const double t = wave_scatter<16>(m);
                const int q = lane >> 2;
                if ((lane & 3) == 0 && q < 14) out[(int64_t)j * 14 + q] = q == 0 ? (double)cnt : t;
            }
        }
        // the group's larger cells; the bounds are the same for every thread
        for (int w = 0; w < CPG; ++w) {
            const int jj = g * CPG + w;
            if (jj >= n_cells) break;
            const int lo = cs[jj], cnt = cs[jj + 1] - lo;
            if (cnt <= MOM_WAVE_MAX) continue;
            double m[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) m[q] = 0.0;
            mom_range<R>(m, v, n, lo + threadIdx.x, (int64_t)lo + cnt, MOM_T);
            const double t = block_sum_scatter<16>(m, red);   // its barriers end the cell
            if (threadIdx.x < 14) out[(int64_t)jj * 14 + threadIdx.x] = threadIdx.x == 0 ? (double)cnt : t;
        }
    }
}

template <typename R>
__global__ void k_unsort_scatter(const R *__restrict__ v, const uint32_t *__restrict__ pid,
                                 const int32_t *__restrict__ cell_of, int64_t n, R *__restrict__ tv,
                                 int32_t *__restrict__ tc)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t d = pid[k];
        if ((int64_t)d >= n) continue;
        tv[d] = v[k];
        tv[n + d] = v[n + k];
        tv[2 * n + d] = v[2 * n + k];
        tc[d] = cell_of[k];
    }
}

template <typename R>
__global__ void k_unsort_copy(R *__restrict__ v, uint32_t *__restrict__ pid, int32_t *__restrict__ cell_of,
                              int64_t n, const R *__restrict__ tv, const int32_t *__restrict__ tc)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        v[k] = tv[k];
        v[n + k] = tv[n + k];
        v[2 * n + k] = tv[2 * n + k];
        cell_of[k] = tc[k];
        pid[k] = (uint32_t)k;
    }
}

// DSMC-Coll step of the electron-heavy collisions C1..C4 for one particle
// per lane (storage order irrelevant: no particle reads another).  The
// decision is taken in binary64 with the operations in the order of the
// definition and no contraction, so it matches a binary64 evaluation
// elsewhere up to the last bit of the exponential.  The cross-section table
// sits in LDS; the breakpoints are shared by the channels, so one segment
// search serves all four.  Since 1 - exp(-x) < x, a draw at or above
// 1.000001 sum_c x_c cannot fall below the cumulative probability: such a
// particle (most of them) is decided without an exponential.  (A binary32
// screen in front of this measured slower.)
__device__ __forceinline__ void dsmc_dir(uint32_t wa, uint32_t wb, double &sx, double &sy, double &sz)
{
#pragma clang fp contract(off)
    const double ct = 1.0 - 2.0 * u01d(wa);
    const double st = sqrt(fmax(0.0, 1.0 - ct * ct));
    const double ph = 2.0 * 3.14159265358979323846 * u01d(wb);
    sx = st * cos(ph);
    sy = st * sin(ph);
    sz = ct;
}

template <typename R>
__global__ __launch_bounds__(256) void k_dsmc(DsmcArgs a, DsmcTable t)
{
#pragma clang fp contract(off)
    __shared__ double s_br[DSMC_MAX_SEG + 1];
    __shared__ double s_co[4 * DSMC_MAX_SEG * 4];
    for (int i = threadIdx.x; i <= t.nseg; i += blockDim.x) s_br[i] = t.breaks[i];
    for (int i = threadIdx.x; i < 16 * t.nseg; i += blockDim.x) s_co[i] = t.coef[i];
    __syncthreads();
    R *vx = (R *)a.v, *vy = vx + a.n, *vz = vy + a.n;
    R *nx = (R *)a.v_new, *ny = nx + a.cap, *nz = ny + a.cap;
    const uint32_t step = (uint32_t)a.step;
    for (int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; l < a.n;
         l += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t p = a.pid[l];
        const int32_t cl = a.cell[l];
        if (cl < 0 || cl >= a.n_cells) {
            atomicOr(&a.dflags->sticky_range, 1);
            continue;
        }
        const double dg = a.ng ? a.ng[cl] : a.ng0;
        const double dm = a.nm ? a.nm[cl] : a.nm0;
        const double x = vx[l], y = vy[l], z = vz[l];
        const double sp2 = x * x + y * y + z * z;
        const double sp = sqrt(sp2);
        const double E = 0.5 * sp2;
        // cross sections: one segment search, four cubics
        int sg = 0;
        while (sg + 1 < t.nseg && E >= s_br[sg + 1]) ++sg;
        double xe = E - s_br[sg];
        const double xmax = s_br[sg + 1] - s_br[sg];
        if (xe > xmax) xe = xmax;
        double sig[4], bound = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double *q = s_co + (c * t.nseg + sg) * 4;
            const double v3 = ((q[3] * xe + q[2]) * xe + q[1]) * xe + q[0];
            sig[c] = E < t.thr[c] ? 0.0 : (v3 > 0.0 ? v3 : 0.0);
            bound += a.dt * sp * sig[c] * (c == 3 ? dm : dg);
        }
        const W4 w = draw4(a.seed, p, step, 6u, 0u);
        const double R0 = u01d(w.x);
        int ch = -1;
        if (R0 < 1.000001 * bound) {
            double cum = 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if (ch < 0) {
                    const double dens = c == 3 ? dm : dg;
                    cum += 1.0 - exp(-a.dt * sp * sig[c] * dens);
                    if (R0 < cum) ch = c;
                }
            }
        }
        if (a.chan_out) a.chan_out[l] = (uint8_t)(ch + 1);
        if (ch < 0) continue;
        double sx, sy, sz, scale;
        dsmc_dir(w.y, w.z, sx, sy, sz);
        if (ch == 0) {
            scale = sp;
            if (sp > 0.0 && t.mass_ratio != 0.0) {
                const double cosx = (x * sx + y * sy + z * sz) / sp;
                scale = sp * sqrt(1.0 - 2.0 * t.mass_ratio * (1.0 - cosx));
            }
        } else if (ch == 2) {
            scale = sqrt(2.0 * (E - t.thr[2]));
        } else {
            const double rem = E - t.thr[ch];
            const double e1 = u01d(w.w) * rem;
            const double e2 = rem - e1;
            scale = sqrt(2.0 * e1);
            const W4 w2 = draw4(a.seed, p, step, 7u, 0u);
            double tx, ty, tz;
            dsmc_dir(w2.y, w2.z, tx, ty, tz);
            const double sc2 = sqrt(2.0 * e2);
            // the new electron: one slot from the shared counter (ionization is rare)
            const unsigned long long k = atomicAdd(a.count, 1ull);
            if (k < (unsigned long long)a.cap) {
                nx[k] = (R)(sc2 * tx);
                ny[k] = (R)(sc2 * ty);
                nz[k] = (R)(sc2 * tz);
                a.pid_new[k] = a.pid_base + p;
                a.cell_new[k] = cl;
            } else {
                atomicOr(&a.dflags->sticky_state, 1);
            }
        }
        vx[l] = (R)(scale * sx);
        vy[l] = (R)(scale * sy);
        vz[l] = (R)(scale * sz);
    }
}

int grid_for(int64_t n, int threads, int cap)
{
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace

int launch_mcc(int dtype, void *v, const uint32_t *pid, int64_t n, uint64_t thr, double mass_ratio,
               uint64_t seed, uint64_t step, uint8_t *cand_out, hipStream_t st)
{
    if (n <= 0) return PIC_OK;
    const int g = grid_for(n, 256, 65536);
    if (dtype == PIC_F32)
        hipLaunchKernelGGL(k_mcc<float>, dim3(g), dim3(256), 0, st, (float *)v, pid, n, thr,
                           mass_ratio, seed, (uint32_t)step, cand_out);
    else
        hipLaunchKernelGGL(k_mcc<double>, dim3(g), dim3(256), 0, st, (double *)v, pid, n, thr,
                           mass_ratio, seed, (uint32_t)step, cand_out);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

int launch_philox(uint64_t seed, uint64_t step, uint32_t domain, uint32_t c3, const uint32_t *c0,
                  int64_t n, uint32_t *out, hipStream_t st)
{
    if (n <= 0) return PIC_OK;
    hipLaunchKernelGGL(k_philox, dim3(grid_for(n, 256, 65536)), dim3(256), 0, st, seed,
                       (uint32_t)step, domain, c3, c0, n, (uint4 *)out);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

int launch_moments(int dtype, const void *v, int64_t n, const int32_t *cell_start,
                   int32_t n_cells, double *out, const int *run_if, int num_cu, hipStream_t st)
{
    const int groups = (n_cells + MOM_T / PIC_WAVE - 1) / (MOM_T / PIC_WAVE);
    const int g = groups < num_cu * 8 ? groups : num_cu * 8;
    if (dtype == PIC_F32)
        hipLaunchKernelGGL(k_moments<float>, dim3(g), dim3(MOM_T), 0, st, (const float *)v, n,
                           cell_start, n_cells, out, run_if);
    else
        hipLaunchKernelGGL(k_moments<double>, dim3(g), dim3(MOM_T), 0, st, (const double *)v, n,
                           cell_start, n_cells, out, run_if);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

int launch_unsort(int dtype, void *v, uint32_t *pid, int32_t *cell_of, int64_t n, void *tmp,
                  hipStream_t st)
{
    if (n <= 0) return PIC_OK;
    const int g = grid_for(n, 256, 65536);
    if (dtype == PIC_F32) {
        float *tv = (float *)tmp;
        int32_t *tc = (int32_t *)(tv + 3 * n);
        hipLaunchKernelGGL(k_unsort_scatter<float>, dim3(g), dim3(256), 0, st, (const float *)v,
                           pid, cell_of, n, tv, tc);
        hipLaunchKernelGGL(k_unsort_copy<float>, dim3(g), dim3(256), 0, st, (float *)v, pid,
                           cell_of, n, (const float *)tv, (const int32_t *)tc);
    } else {
        double *tv = (double *)tmp;
        int32_t *tc = (int32_t *)(tv + 3 * n);
        hipLaunchKernelGGL(k_unsort_scatter<double>, dim3(g), dim3(256), 0, st, (const double *)v,
                           pid, cell_of, n, tv, tc);
        hipLaunchKernelGGL(k_unsort_copy<double>, dim3(g), dim3(256), 0, st, (double *)v, pid,
                           cell_of, n, (const double *)tv, (const int32_t *)tc);
    }
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

int launch_dsmc(int dtype, const DsmcArgs &a, const DsmcTable &t, hipStream_t st)
{
    if (a.n <= 0) return PIC_OK;
    const int g = grid_for(a.n, 256, 65536);
    if (dtype == PIC_F32)
        hipLaunchKernelGGL(k_dsmc<float>, dim3(g), dim3(256), 0, st, a, t);
    else
        hipLaunchKernelGGL(k_dsmc<double>, dim3(g), dim3(256), 0, st, a, t);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

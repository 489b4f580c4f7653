// Particle-to-cell sums (section "Particle-to-Cell", steps S3a-S3b of the
// PIC scheme table): V^j = sum over the particles l of cell j of a vector
// V_l of nq per-particle quantities, particles in any order, binary64
// accumulation.
//
// The paper reduces with atomics straight into per-cell accumulators, split
// into sub-cell copies V^{jm} when cells are crowded, and sums the copies
// afterwards.  Here, when the nq M accumulators fit in LDS, every workgroup
// keeps a private copy there (the sub-cell copies become per-workgroup LDS
// copies: LDS atomics, no global traffic but the final partials), and a
// second pass adds the workgroups' partials in a fixed order.  Larger grids
// take the paper's form: global binary64 atomics into m copies, then their
// sum.  A wave whose particles all lie in one cell (the storage the collision
// step leaves is cell-sorted) adds its values in registers first and issues
// one atomic per quantity.
#include "pic_internal.hpp"

#define HIP_OK(x) do { if ((x) != hipSuccess) return PIC_ERR_HIP; } while (0)

namespace {

constexpr int P2C_LDS_T = 1024;
constexpr int P2C_GLB_T = 256;
constexpr size_t P2C_LDS_MAX = 128 * 1024;   // bytes of LDS accumulators per workgroup

__device__ __forceinline__ double wave_sum_d(double x)
{
#pragma unroll
    for (int o = PIC_WAVE / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, PIC_WAVE);
    return x;
}

// One slice of particles into the accumulators acc[c * NQ + k] (LDS or
// global).  Each thread keeps running sums while its particles stay in one
// cell (in the cell-sorted storage a thread's particles, blockDim apart,
// mostly share a cell) and adds them when the cell changes; a wave whose
// flushing lanes all hold the same cell adds in registers and issues one
// atomic per quantity.  Four iterations' loads are issued before any is
// used (eight in the LDS form).  Whole waves take part in every iteration so that the ballots see
// every lane.
template <int NQ, bool LDS>
__device__ __forceinline__ void p2c_flush(bool fl, int32_t cur, const double (&run)[NQ], double *acc)
{
    const uint64_t fm = __ballot(fl);
    if (!fm) return;
    const int leader = __ffsll((unsigned long long)fm) - 1;
    const int32_t c0 = __shfl(cur, leader, PIC_WAVE);
    if (__ballot(fl && cur != c0) == 0) {
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            const double s = wave_sum_d(fl ? run[k] : 0.0);
            if ((int)(threadIdx.x & (PIC_WAVE - 1)) == leader) {
                if (LDS) atomicAdd(&acc[c0 * NQ + k], s);
                else unsafeAtomicAdd(&acc[(int64_t)c0 * NQ + k], s);
            }
        }
    } else if (fl) {
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            if (LDS) atomicAdd(&acc[cur * NQ + k], run[k]);
            else unsafeAtomicAdd(&acc[(int64_t)cur * NQ + k], run[k]);
        }
    }
}

template <typename R, int NQ, bool LDS>
__device__ __forceinline__ void p2c_slice(const R *__restrict__ q, const int32_t *__restrict__ cell_of, int64_t n,
                                          int32_t M, int64_t start, int64_t end, int64_t step, double *acc,
                                          DevFlags *f)
{
    constexpr int U = LDS ? 8 : 4;   // one 16-wave workgroup per CU in the LDS form
    bool bad_any = false;
    int32_t cur = -1;   // cell of the running sums, -1: none yet
    double run[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) run[k] = 0.0;
    for (int64_t i0 = start; i0 < end; i0 += U * step) {
        int32_t c[U];
        R x[U][NQ];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            // past the end: reload the last particle (masked below), so the
            // loads need no branch and all of them are in flight together
            int64_t l = i0 + u * step + threadIdx.x;
            l = l < end ? l : end - 1;
            c[u] = cell_of[l];
#pragma unroll
            for (int k = 0; k < NQ; ++k) x[u][k] = q[(int64_t)k * n + l];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool valid = i0 + u * step + threadIdx.x < end;
            const bool bad = valid && (c[u] < 0 || c[u] >= M);   // masks the reloaded ones too
            bad_any |= bad;
            const bool ok = valid && !bad;
            const bool fl = ok && cur >= 0 && c[u] != cur;   // leaving a cell
            p2c_flush<NQ, LDS>(fl, cur, run, acc);
            if (ok) {
                const bool fresh = cur != c[u];
#pragma unroll
                for (int k = 0; k < NQ; ++k) run[k] = (fresh ? 0.0 : run[k]) + (double)x[u][k];
                cur = c[u];
            }
        }
    }
    p2c_flush<NQ, LDS>(cur >= 0, cur, run, acc);
    if (__ballot(bad_any) && (threadIdx.x & (PIC_WAVE - 1)) == 0) {
        atomicOr(&f->range_err, 1);
        atomicOr(&f->sticky_range, 1);
    }
}

// Per-workgroup LDS copy; the workgroup's partial sums go to part[blockIdx].
template <typename R, int NQ>
__global__ __launch_bounds__(P2C_LDS_T) void k_p2c_lds(const R *__restrict__ q, const int32_t *__restrict__ cell_of,
                                                       int64_t n, int32_t M, int64_t chunk,
                                                       double *__restrict__ part, DevFlags *f)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double *acc = (double *)smem;
    const int W = M * NQ;
    for (int j = threadIdx.x; j < W; j += P2C_LDS_T) acc[j] = 0.0;
    __syncthreads();
    const int64_t start = blockIdx.x * chunk;
    const int64_t end = start + chunk < n ? start + chunk : n;
    p2c_slice<R, NQ, true>(q, cell_of, n, M, start, end, P2C_LDS_T, acc, f);
    __syncthreads();
    double *out = part + (size_t)blockIdx.x * W;
    for (int j = threadIdx.x; j < W; j += P2C_LDS_T) out[j] = acc[j];
}

// Global binary64 atomics into copy (blockIdx mod m) of the accumulators.
template <typename R, int NQ>
__global__ __launch_bounds__(P2C_GLB_T) void k_p2c_global(const R *__restrict__ q,
                                                          const int32_t *__restrict__ cell_of, int64_t n,
                                                          int32_t M, int64_t chunk, int m,
                                                          double *__restrict__ copies, DevFlags *f)
{
    const int64_t start = blockIdx.x * chunk;
    const int64_t end = start + chunk < n ? start + chunk : n;
    double *acc = copies + (size_t)(blockIdx.x % m) * M * NQ;
    p2c_slice<R, NQ, false>(q, cell_of, n, M, start, end, P2C_GLB_T, acc, f);
}

__global__ void k_p2c_zero(double *__restrict__ p, int64_t count)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// out[j] = sum over s < copies of part[s * W + j] in a fixed order: wave w
// of the workgroup adds the copies s = w mod 4, then the four partials are
// added.
__global__ __launch_bounds__(256) void k_p2c_reduce(const double *__restrict__ part, int copies, int64_t W,
                                                    double *__restrict__ out)
{
    __shared__ double red[4][PIC_WAVE];
    const int lane = threadIdx.x & (PIC_WAVE - 1), w = threadIdx.x / PIC_WAVE;
    for (int64_t j0 = blockIdx.x * (int64_t)PIC_WAVE; j0 < W; j0 += (int64_t)gridDim.x * PIC_WAVE) {
        const int64_t j = j0 + lane;
        double s = 0.0;
        if (j < W)
            for (int c = w; c < copies; c += 4) s += part[(size_t)c * W + j];
        red[w][lane] = s;
        __syncthreads();
        if (w == 0 && j < W) out[j] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
        __syncthreads();
    }
}

struct P2cPlan {
    bool lds;
    int G, m;          // workgroups; accumulator copies (global form)
    int64_t chunk;
};

P2cPlan p2c_plan(int64_t n, int32_t M, int nq, int num_cu)
{
    P2cPlan p;
    const size_t bytes = (size_t)M * nq * 8;
    p.lds = bytes <= P2C_LDS_MAX;
    const int T = p.lds ? P2C_LDS_T : P2C_GLB_T;
    int per_cu = p.lds ? (int)(160 * 1024 / bytes) : 8;
    if (per_cu < 1) per_cu = 1;
    if (per_cu > 2) per_cu = p.lds ? 2 : per_cu;   // 2 x 1024 threads fill a CU
    int64_t G = (int64_t)num_cu * per_cu;
    const int64_t need = (n + T - 1) / T;
    if (G > need) G = need;
    if (G < 1) G = 1;
    p.chunk = (n + G - 1) / G;
    p.chunk = (p.chunk + T - 1) / T * T;   // whole-workgroup steps
    if (p.chunk < T) p.chunk = T;
    p.G = (int)((n + p.chunk - 1) / p.chunk);
    if (p.G < 1) p.G = 1;
    // crowded cells: more copies (the paper's sub-cells), at most 8
    const int64_t per_cell = n / (M > 0 ? M : 1);
    int m = (int)((per_cell + 1023) / 1024);
    p.m = p.lds ? p.G : (m < 1 ? 1 : m > 8 ? 8 : m);
    return p;
}

template <typename R, int NQ>
int launch_p2c_t(const void *q, const int32_t *cell_of, int64_t n, int32_t M, double *out, void *ws,
                 DevFlags *f, int num_cu, hipStream_t st)
{
    const P2cPlan p = p2c_plan(n, M, NQ, num_cu);
    const int64_t W = (int64_t)M * NQ;
    double *part = (double *)ws;
    const int rg = (int)((W + 255) / 256 < 4096 ? (W + 255) / 256 : 4096);
    const int rr = (int)((W + PIC_WAVE - 1) / PIC_WAVE < 4096 ? (W + PIC_WAVE - 1) / PIC_WAVE : 4096);
    if (n > 0 && p.lds) {
        const size_t lds = (size_t)W * 8;
        auto kern = k_p2c_lds<R, NQ>;
        HIP_OK(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(kern, dim3(p.G), dim3(P2C_LDS_T), lds, st, (const R *)q, cell_of, n, M, p.chunk,
                           part, f);
    } else if (n > 0) {
        hipLaunchKernelGGL(k_p2c_zero, dim3(rg), dim3(256), 0, st, part, (int64_t)p.m * W);
        hipLaunchKernelGGL((k_p2c_global<R, NQ>), dim3(p.G), dim3(P2C_GLB_T), 0, st, (const R *)q, cell_of, n, M,
                           p.chunk, p.m, part, f);
    }
    hipLaunchKernelGGL(k_p2c_reduce, dim3(rr), dim3(256), 0, st, (const double *)part, n > 0 ? p.m : 0, W, out);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

template <typename R>
int launch_p2c_r(int nq, const void *q, const int32_t *cell_of, int64_t n, int32_t M, double *out, void *ws,
                 DevFlags *f, int num_cu, hipStream_t st)
{
    switch (nq) {
    case 1: return launch_p2c_t<R, 1>(q, cell_of, n, M, out, ws, f, num_cu, st);
    case 2: return launch_p2c_t<R, 2>(q, cell_of, n, M, out, ws, f, num_cu, st);
    case 3: return launch_p2c_t<R, 3>(q, cell_of, n, M, out, ws, f, num_cu, st);
    default: return launch_p2c_t<R, 4>(q, cell_of, n, M, out, ws, f, num_cu, st);
    }
}

}  // namespace

size_t p2c_ws_bytes(int64_t n, int32_t M, int nq, int num_cu)
{
    const P2cPlan p = p2c_plan(n, M, nq, num_cu);
    return (size_t)p.m * M * nq * 8 + 256;
}

int launch_p2c(int dtype, int nq, const void *q, const int32_t *cell_of, int64_t n, int32_t M, double *out,
               void *ws, DevFlags *f, int num_cu, hipStream_t st)
{
    if (dtype == PIC_F32) return launch_p2c_r<float>(nq, q, cell_of, n, M, out, ws, f, num_cu, st);
    return launch_p2c_r<double>(nq, q, cell_of, n, M, out, ws, f, num_cu, st);
}

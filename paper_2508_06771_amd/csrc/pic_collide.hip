// pic_collide.hip -- the per-cell Coulomb collision pass (Table "Coulombic
// Collision Steps", CCS3-CCS5) with the null-collision step, the per-cell
// FP64 conservation sums and the moment sums fused into the same pass.
//
// The paper keeps particles unsorted, builds index lists and then gathers
// velocities at random addresses for every pair ("6 reads and 6 writes" per
// pair, non-coalesced, the bulk of its Coulomb time).  Here storage is in
// cell order, so one workgroup owns a cell's contiguous range: velocities and
// ids are streamed in and out coalesced exactly once, the random pairing is a
// sort of the cell's keys in LDS, and partners meet through LDS.  The random
// numbers come from Philox in registers (no pre-generated arrays).
//
// Per cell (n members, all in registers: K per thread):
//   1. load pid, v; one Philox4x32-10 call per particle (domain 0):
//      word0 pairing key, word1 null-collision candidate, words 2-3 for the pair
//   2. sort by (key, pid) with an LDS bucket sort: bucket = (key * nb) >> 32
//      is monotone in key, so buckets in order and (key, pid) order inside a
//      bucket (expected 2 members) give the full order
//   3. pairs (2i, 2i+1): second members post (v, word2) in LDS, first members
//      apply the Takizuka & Abe rotation and post the half change back
//   4. optional FP64 momentum/energy correction, null-collision scattering of
//      candidates, optional moment sums; store v.
//
// Cells larger than the biggest LDS class take the "huge" path below, the same
// algorithm with its per-cell arrays in global scratch indexed by slot.
#include <float.h>

#include <type_traits>

#include "pic_internal.hpp"

#define HIP_OK(x) do { if ((x) != hipSuccess) return PIC_ERR_HIP; } while (0)

namespace {

constexpr double PI_D = 3.14159265358979323846;

// Half of the Takizuka & Abe velocity change of the pair (a, b) with
// relative velocity u = v_a - v_b.  C = 8 pi n lnL dt (so s^2 = C / |u|^3);
// U1, U2 (words 2, 3 of a) give z by Box-Muller, U3 (word 2 of b) the
// azimuth.  The rotation keeps |u|: u' = u cos T + |u| sin T (cos P e1 + sin P e2).
// The standard normal deviate of the pair from words 2, 3 of its first member
// (Box-Muller, cosine branch; the hardware log is base 2 and the cosine takes
// revolutions; the hardware square root, within 1 ulp, where the correctly
// rounded one costs about 16 more instructions).
__device__ __forceinline__ float ta_z(uint32_t wa2, uint32_t wa3)
{
    return __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u01f(wa2))) *
           __builtin_amdgcn_cosf(u01f(wa3));
}

// The same from the deviate z already drawn.
__device__ __forceinline__ void ta_half_z(float ux, float uy, float uz, float C, float z,
                                          uint32_t wb2, float &hx, float &hy, float &hz)
{
    const float uu = ux * ux + uy * uy + uz * uz;
    hx = hy = hz = 0.0f;
    if (!(uu >= FLT_MIN)) return;   // u = 0 (or below the normal range): no change
    const float rinv = __builtin_amdgcn_rsqf(uu);     // 1 / |u|
    const float um = uu * rinv;                        // |u|
    const float s = __builtin_amdgcn_sqrtf(C * rinv * rinv * rinv);
    const float d = s * z;
    // sin T = 2d / (1 + d^2), 1 - cos T = 2 d^2 / (1 + d^2); for |d| > 1 the
    // same ratios in t = 1/d avoid overflow of d^2.
    float sin_t, omc;
    if (fabsf(d) <= 1.0f) {
        const float inv = __builtin_amdgcn_rcpf(1.0f + d * d);
        sin_t = 2.0f * d * inv;
        omc = 2.0f * d * d * inv;
    } else {
        const float t = __builtin_amdgcn_rcpf(d);
        const float inv = __builtin_amdgcn_rcpf(1.0f + t * t);
        sin_t = 2.0f * t * inv;
        omc = 2.0f * inv;
    }
    const float u3 = u01f(wb2);
    const float cp = __builtin_amdgcn_cosf(u3), sp = __builtin_amdgcn_sinf(u3);  // revolutions
    const float up2 = ux * ux + uy * uy;
    float dx, dy, dz;
    if (up2 > 0.0f) {
        const float upinv = __builtin_amdgcn_rsqf(up2);
        const float up = up2 * upinv;
        const float a = uz * sin_t * cp;
        const float b = um * sin_t * sp;
        dx = (ux * upinv) * a - (uy * upinv) * b - ux * omc;
        dy = (uy * upinv) * a + (ux * upinv) * b - uy * omc;
        dz = -up * sin_t * cp - uz * omc;
    } else {
        dx = um * sin_t * cp;
        dy = um * sin_t * sp;
        dz = -uz * omc;
    }
    hx = 0.5f * dx;
    hy = 0.5f * dy;
    hz = 0.5f * dz;
}

__device__ __forceinline__ void ta_half(float ux, float uy, float uz, float C, uint32_t wa2,
                                        uint32_t wa3, uint32_t wb2, float &hx, float &hy,
                                        float &hz)
{
    ta_half_z(ux, uy, uz, C, ta_z(wa2, wa3), wb2, hx, hy, hz);
}

__device__ __forceinline__ void ta_half(double ux, double uy, double uz, double C, uint32_t wa2,
                                        uint32_t wa3, uint32_t wb2, double &hx, double &hy,
                                        double &hz)
{
#pragma clang fp contract(off)
    const double uu = ux * ux + uy * uy + uz * uz;
    hx = hy = hz = 0.0;
    if (uu == 0.0) return;
    const double um = sqrt(uu);
    const double uperp = sqrt(ux * ux + uy * uy);
    const double z = sqrt(-2.0 * log(u01d(wa2))) * cos(2.0 * PI_D * u01d(wa3));
    const double s2 = C / (um * um * um);
    const double d = sqrt(s2) * z;
    double sin_t, omc;
    if (fabs(d) <= 1e150) {
        sin_t = 2.0 * d / (1.0 + d * d);
        omc = 2.0 * d * d / (1.0 + d * d);
    } else {
        sin_t = 2.0 / d;
        omc = 2.0;
    }
    const double phi = 2.0 * PI_D * u01d(wb2);
    const double cp = cos(phi), sp = sin(phi);
    double dx, dy, dz;
    if (uperp > 0.0) {
        dx = (ux / uperp) * uz * sin_t * cp - (uy / uperp) * um * sin_t * sp - ux * omc;
        dy = (uy / uperp) * uz * sin_t * cp + (ux / uperp) * um * sin_t * sp - uy * omc;
        dz = -uperp * sin_t * cp - uz * omc;
    } else {
        dx = um * sin_t * cp;
        dy = um * sin_t * sp;
        dz = -uz * omc;
    }
    hx = 0.5 * dx;
    hy = 0.5 * dy;
    hz = 0.5 * dz;
}

template <typename R>
__device__ __forceinline__ void mcc_scatter(R &vx, R &vy, R &vz, uint32_t pid, uint64_t seed,
                                            uint32_t step, double mass_ratio)
{
    scatter_dir(vx, vy, vz, draw4(seed, pid, step, 1u, 0u), mass_ratio);
}

__device__ __forceinline__ uint64_t read_step(const CollideArgs &a)
{
    return a.step_dev ? *a.step_dev : a.step;
}

__device__ __forceinline__ double cell_C(const CollideArgs &a, int cell)
{
    const double dens = a.density ? a.density[cell] : 1.0;
    const double dts = a.dt_scale ? a.dt_scale[cell] : 1.0;
    return 8.0 * PI_D * dens * a.lnL * a.dt * dts;
}

__device__ __forceinline__ bool gated_off(const CollideArgs &a)
{
    if (a.dflags->range_err) return true;
    if ((a.flags & PIC_ASSUME_SORTED) && a.dflags->unsorted) return true;
    return false;
}

// Variants compiled per kernel: which optional parts of the pass exist.
enum { F_MCC = 1, F_CONS = 2, F_MOM = 4, F_PAIRS = 8, F_WT = 16, F_NANBU = 32, F_TRIP = 64 };

// Variable-weight rule for the pair (a, b) with half change h (a += h,
// b -= h in the uniform step): the member of smaller weight always takes its
// half, the other one iff U4 * w_heavy < w_light in binary64, U4 = U(word 3 of
// b's domain-0 draw).  Equal weights: both take it.
template <typename R>
__device__ __forceinline__ void weight_rule(R wa, R wb, uint32_t w3b, bool &take_a, bool &take_b)
{
    take_a = take_b = true;
    if (wa != wb) {
        const double U4 = u01d(w3b);
        if (wa > wb) take_a = U4 * (double)wa < (double)wb;
        else take_b = U4 * (double)wb < (double)wa;
    }
}

// Pair-major exchange records.  In each round the members whose sorted
// position falls in the round post their velocity and word 2 at that
// position (first members also word 3, at the pair index); one thread per
// pair applies the Takizuka & Abe rotation and writes both new velocities
// back in place; each member then reads its own record.
template <typename R> struct Rec;
template <> struct __align__(16) Rec<float> { float x, y, z; uint32_t w2; };
template <> struct __align__(16) Rec<double> { double x, y, z; uint32_t w2, pad; };

// Dynamic LDS a cell pass may use (the static part is below 4 KB).
constexpr size_t LDS_DYN_LIMIT = 152 * 1024;

// Layout of one exchange round of P positions: P + 2 records (two beyond P
// for an odd cell's triplet that straddles the end of the round), the first
// members' word 3 per pair, and with weights the second members' word 3 and
// the weight per position, with Nanbu's operator or the triplet the member
// index per position.
template <typename R, int F>
struct ExchLayout {
    static constexpr bool WT = (F & F_WT) != 0;
    static constexpr bool SLOT = (F & (F_NANBU | F_TRIP)) != 0;
    __host__ __device__ static constexpr size_t bytes(uint32_t P)
    {
        size_t b = ((size_t)P + 2) * sizeof(Rec<R>) + ((size_t)P / 2 + 1) * 4;
        if (WT) b += ((size_t)P / 2 + 1) * 4 + ((size_t)P + 2) * sizeof(R);
        if (SLOT) b += ((size_t)P + 2) * 2;
        return (b + 15) & ~(size_t)15;
    }
};

// Positions per exchange round: the whole cell when its records fit.
template <typename R, int F = 0>
__host__ __device__ constexpr uint32_t round_positions(int cap)
{
    const uint32_t want = (uint32_t)(((size_t)cap + 1) & ~(size_t)1);
    uint32_t P = want;
    while (P > 64 && ExchLayout<R, F>::bytes(P) > LDS_DYN_LIMIT) P -= 64;
    return P;
}

template <typename R, int F = 0>
__host__ __device__ constexpr size_t lds_bytes(int cap)
{
    const size_t ex = ExchLayout<R, F>::bytes(round_positions<R, F>(cap));
    const size_t s = sort_bytes(cap);
    return s > ex ? s : ex;
}

// Nanbu's deflection of the pair (a, b), a the member in the lower storage
// slot: 1 - cos chi from Nanbu's distribution with U = U(word 2 of a) and
// A(s), s twice the Takizuka & Abe variance (C / |u|^3, C = 8 pi n lnL dt);
// azimuth 2 pi U(word 2 of b); rotation and halves as in Takizuka & Abe.
// Binary64 computes the oracle's steps; binary32 its own (see nb_A).
template <typename R>
__device__ __forceinline__ void nanbu_half(R ux, R uy, R uz, R C, uint32_t wa2, uint32_t wb2, R &hx,
                                           R &hy, R &hz)
{
#pragma clang fp contract(off)
    const double PI = 3.14159265358979323846;
    hx = hy = hz = (R)0;
    const R uu = ux * ux + uy * uy + uz * uz;
    if (uu == (R)0) return;
    const R um = sqrt(uu), uperp = sqrt(ux * ux + uy * uy);
    const R s = (R)2 * nb_div(C, um * um * um);
    const R U = sizeof(R) == 4 ? (R)u01f(wa2) : (R)u01d(wa2);
    const R omc = nb_omc(nb_A(s), U);
    const R sin_t = sqrt(omc * ((R)2 - omc));
    const R phi = (R)(2.0 * PI) * (sizeof(R) == 4 ? (R)u01f(wb2) : (R)u01d(wb2));
    const R cphi = cos(phi), sphi = sin(phi);
    R dx, dy, dz;
    if (uperp > (R)0) {
        const R ex = nb_div(ux, uperp), ey = nb_div(uy, uperp);
        dx = ex * uz * sin_t * cphi - ey * um * sin_t * sphi - ux * omc;
        dy = ey * uz * sin_t * cphi + ex * um * sin_t * sphi - uy * omc;
        dz = -uperp * sin_t * cphi - uz * omc;
    } else {
        dx = um * sin_t * cphi;
        dy = um * sin_t * sphi;
        dz = -uz * omc;
    }
    hx = (R)0.5 * dx;
    hy = (R)0.5 * dy;
    hz = (R)0.5 * dz;
}

// Takizuka & Abe's triplet for an odd cell: the members p0 p1 p2 (the last
// three in pairing order) collide pairwise at dt/2 in the order (p0, p1),
// (p1, p2), (p2, p0), each on the velocities the previous one left, with the
// uniforms of Philox domains 0, 4 and 5.  In place on x, y, z.
template <typename R>
__device__ __forceinline__ void triplet_collide(R (&x)[3], R (&y)[3], R (&z)[3], const uint32_t (&pd)[3],
                                                R Ch, uint64_t seed, uint32_t step)
{
    const uint32_t dom[3] = {0u, 4u, 5u};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int i = c, k = (c + 1) % 3;
        const W4 wa = draw4(seed, pd[i], step, dom[c], 0u);
        const W4 wb = draw4(seed, pd[k], step, dom[c], 0u);
        R hx, hy, hz;
        ta_half(x[i] - x[k], y[i] - y[k], z[i] - z[k], Ch, wa.z, wa.w, wb.z, hx, hy, hz);
        x[i] += hx;
        y[i] += hy;
        z[i] += hz;
        x[k] -= hx;
        y[k] -= hy;
        z[k] -= hz;
    }
}

// ------------------------------------------------------------ LDS-class pass
// Adds the 14 moment terms of v to m[0..13] (layout of pic_cell_moments:
// count, sum v, the second-order products, sum |v|^2 v, sum |v|^4).
__device__ __forceinline__ void moment_terms(double (&m)[16], double x, double y, double z)
{
    const double q2 = x * x + y * y + z * z;
    m[0] += 1.0;
    m[1] += x; m[2] += y; m[3] += z;
    m[4] += x * x; m[5] += y * y; m[6] += z * z;
    m[7] += x * y; m[8] += x * z; m[9] += y * z;
    m[10] += q2 * x; m[11] += q2 * y; m[12] += q2 * z;
    m[13] += q2 * q2;
}

// The 14 moment sums of the pass's members (layout of pic_cell_moments): four
// wave reduce-scatters of 4 values (so at most 4 accumulators are live), each
// into its own quarter of red, then one cross-wave pass.  The count is n.
// red: 16 doubles per wave.  Contains the barriers; threads 0..13 write.
template <typename R, int T, int K>
__device__ __forceinline__ void cell_moments_out(double *out, const R (&vx)[K], const R (&vy)[K],
                                                 const R (&vz)[K], int n, double *red)
{
    constexpr int NW = T / PIC_WAVE;
#pragma unroll
    for (int part = 0; part < 4; ++part) {
        double h[4] = {0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (threadIdx.x + k * T < n) {
                const double x = vx[k], y = vy[k], z = vz[k];
                if (part == 0) {
                    h[0] += x; h[1] += y; h[2] += z; h[3] += x * x;
                } else if (part == 1) {
                    h[0] += y * y; h[1] += z * z; h[2] += x * y; h[3] += x * z;
                } else {
                    const double q2 = x * x + y * y + z * z;
                    if (part == 2) {
                        h[0] += y * z; h[1] += q2 * x; h[2] += q2 * y; h[3] += q2 * z;
                    } else {
                        h[0] += q2 * q2;
                    }
                }
            }
        }
        wave_scatter_to<4>(h, red + part * 4 * NW);
    }
    __syncthreads();
    if (threadIdx.x < 13) {
        const double *r = red + (threadIdx.x >> 2) * 4 * NW + (threadIdx.x & 3);
        double t = 0.0;
        for (int w = 0; w < NW; ++w) t += r[w * 4];
        out[1 + threadIdx.x] = t;
    } else if (threadIdx.x == 13) {
        out[0] = (double)n;
    }
    __syncthreads();
}

template <typename R, int T, int K, int F>
__device__ __forceinline__ void cell_pass(const CollideArgs &a, int cell, unsigned char *smem, double *red,
                          uint32_t *wtot, double *s_before)
{
    constexpr bool PAIRS = (F & F_PAIRS) != 0;
    constexpr bool MCC = (F & F_MCC) != 0;
    constexpr bool CONS = (F & F_CONS) != 0;
    constexpr bool MOM = (F & F_MOM) != 0;
    constexpr bool WT = (F & F_WT) != 0;
    constexpr bool NANBU = (F & F_NANBU) != 0;
    constexpr bool TRIP = (F & F_TRIP) != 0;
    constexpr int CAP = T * K;
    const int lo = a.cell_start[cell];
    const int n = a.cell_start[cell + 1] - lo;
    const uint32_t step = (uint32_t)read_step(a);
    const bool coul = n >= 2;
    R *vx_g = (R *)a.v + lo;
    R *vy_g = (R *)a.v + a.n + lo;
    R *vz_g = (R *)a.v + 2 * a.n + lo;
    const uint32_t *pid_c = a.pid + lo;

    const SortLDS<T, CAP> L(smem);

    R vx[K], vy[K], vz[K];
    uint32_t w2[K], w3[K], pos[K];
    uint32_t cand = 0;

    const uint32_t bits = sort_bits(n);
    // every load of the thread is issued before any is used, so they are in
    // flight together and overlap the clearing of the counters (pos holds
    // the pid until the key is counted)
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = threadIdx.x + k * T;
        if (i < n) {
            pos[k] = pid_c[i];
            if (!PAIRS) {
                vx[k] = vx_g[i];
                vy[k] = vy_g[i];
                vz[k] = vz_g[i];
            }
        }
    }
    L.clear();
    __syncthreads();
    {
        // one Philox call per particle, and the bucket count of its key with
        // its arrival rank
        double before[4] = {0, 0, 0, 0};   // sum v, sum |v|^2
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = threadIdx.x + k * T;
            if (i < n) {
                const W4 w = draw4(a.seed, pos[k], step, 0u, 0u);
                w2[k] = w.z;
                w3[k] = w.w;
                if (MCC && (uint64_t)w.y < a.mcc_thr) cand |= 1u << k;
                pos[k] = L.count(i, w.x, bits);
                if (CONS) {
                    const double x = vx[k], y = vy[k], z = vz[k];
                    before[0] += x;
                    before[1] += y;
                    before[2] += z;
                    before[3] += x * x + y * y + z * z;
                }
            }
        }
        if constexpr (CONS) {
            const double t = block_sum_scatter<4>(before, red);   // contains the barriers
            if (threadIdx.x < 4) s_before[threadIdx.x] = t;
        }
    }
    __syncthreads();

    if (coul || PAIRS) rank_in_lds<T, K, CAP>(pos, n, bits, L, pid_c, wtot);

    if (PAIRS) {
        // sorted[] and partner[] for the test export
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = threadIdx.x + k * T;
            if (i < n) {
                L.lst[pos[k]] = (uint16_t)i;
                a.sorted_out[lo + pos[k]] = lo + i;
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = threadIdx.x + k * T;
            if (i < n) {
                const uint32_t q = pos[k] ^ 1u;
                a.partner_out[lo + i] = (q < (uint32_t)n) ? lo + (int)L.lst[q] : -1;
            }
        }
        __syncthreads();
        return;
    }

    if (coul) {
        const R C = (R)cell_C(a, cell);
        const uint32_t np2 = (uint32_t)n & ~1u;     // positions with a partner
        // with the triplet, an odd cell's last three positions form it
        const uint32_t tstart = (TRIP && (n & 1) && n >= 3) ? (uint32_t)n - 3u : np2;
        const uint32_t npost = tstart < np2 ? (uint32_t)n : np2;   // positions with records
        constexpr uint32_t P = round_positions<R, F>(CAP);
        Rec<R> *rec = (Rec<R> *)smem;
        uint32_t *w3s = (uint32_t *)(rec + P + 2);
        // with weights: the second member's word 3 per pair, the weight per position
        uint32_t *w3b = w3s + P / 2 + 1;
        R *wts = (R *)(w3b + (WT ? P / 2 + 1 : 0));
        // with Nanbu's operator or the triplet: the member index per position
        uint16_t *slt = (uint16_t *)(wts + (WT ? P + 2 : 0));
        const R *w_c = (const R *)a.w + lo;
        for (uint32_t base = 0; base < npost; base += P) {
            // a member posts in the round of its position; the triplet's three
            // in the round holding its start
            const bool tri_here = tstart < npost && tstart >= base && tstart - base < P;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int i = threadIdx.x + k * T;
                const uint32_t q = pos[k] - base;
                const bool mine = pos[k] < tstart ? q < P : (pos[k] < npost && tri_here);
                if (i < n && mine) {
                    Rec<R> e;
                    e.x = vx[k];
                    e.y = vy[k];
                    e.z = vz[k];
                    e.w2 = w2[k];
                    rec[q] = e;
                    if (!(q & 1u)) w3s[q >> 1] = w3[k];
                    if constexpr (WT) {
                        if (q & 1u) w3b[q >> 1] = w3[k];
                        wts[q] = w_c[i];
                    }
                    if constexpr (NANBU || TRIP) slt[q] = (uint16_t)i;
                }
            }
            __syncthreads();
            const uint32_t lim = min(base + P, tstart);
            const uint32_t m = lim > base ? (lim - base) / 2 : 0u;
            for (uint32_t j = threadIdx.x; j < m; j += T) {
                Rec<R> A = rec[2 * j], B = rec[2 * j + 1];
                R hx, hy, hz;
                bool ta = true, tb = true;
                if constexpr (NANBU) {
                    // the member in the lower storage slot is the operator's first
                    if (slt[2 * j] < slt[2 * j + 1]) {
                        nanbu_half<R>(A.x - B.x, A.y - B.y, A.z - B.z, C, A.w2, B.w2, hx, hy, hz);
                    } else {
                        nanbu_half<R>(B.x - A.x, B.y - A.y, B.z - A.z, C, B.w2, A.w2, hx, hy, hz);
                        hx = -hx;
                        hy = -hy;
                        hz = -hz;
                    }
                } else {
                    ta_half(A.x - B.x, A.y - B.y, A.z - B.z, C, A.w2, w3s[j], B.w2, hx, hy, hz);
                    if constexpr (WT) weight_rule<R>(wts[2 * j], wts[2 * j + 1], w3b[j], ta, tb);
                }
                if (ta) {
                    A.x += hx;
                    A.y += hy;
                    A.z += hz;
                }
                if (tb) {
                    B.x -= hx;
                    B.y -= hy;
                    B.z -= hz;
                }
                rec[2 * j] = A;
                rec[2 * j + 1] = B;
            }
            if constexpr (TRIP) {
                if (tri_here && threadIdx.x == 0) {
                    const uint32_t q0 = tstart - base;
                    R x[3], y[3], z[3];
                    uint32_t pd[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const Rec<R> e = rec[q0 + c];
                        x[c] = e.x;
                        y[c] = e.y;
                        z[c] = e.z;
                        pd[c] = pid_c[slt[q0 + c]];
                    }
                    const double dens = a.density ? a.density[cell] : 1.0;
                    triplet_collide<R>(x, y, z, pd, (R)(8.0 * PI_D * dens * a.lnL * (0.5 * a.dt)),
                                       a.seed, step);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        Rec<R> e = rec[q0 + c];
                        e.x = x[c];
                        e.y = y[c];
                        e.z = z[c];
                        rec[q0 + c] = e;
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int i = threadIdx.x + k * T;
                const uint32_t q = pos[k] - base;
                const bool mine = pos[k] < tstart ? q < P : (pos[k] < npost && tri_here);
                if (i < n && mine) {
                    const Rec<R> e = rec[q];
                    vx[k] = e.x;
                    vy[k] = e.y;
                    vz[k] = e.z;
                }
            }
            if (base + P < npost) __syncthreads();
        }

        if constexpr (CONS) {
            double after[4] = {0, 0, 0, 0};
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int i = threadIdx.x + k * T;
                if (i < n) {
                    const double x = vx[k], y = vy[k], z = vz[k];
                    after[0] += x;
                    after[1] += y;
                    after[2] += z;
                    after[3] += x * x + y * y + z * z;
                }
            }
            block_sum_bcast<4>(after, red);
            const Correction cr = make_correction((double)n, s_before, after,
                                                  a.debt ? a.debt + (int64_t)cell * 4 : nullptr);
            if (cr.ok) {
                double real[4] = {0, 0, 0, 0};
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const int i = threadIdx.x + k * T;
                    if (i < n) {
                        vx[k] = (R)(cr.Vt[0] + cr.al * ((double)vx[k] - cr.Vn[0]));
                        vy[k] = (R)(cr.Vt[1] + cr.al * ((double)vy[k] - cr.Vn[1]));
                        vz[k] = (R)(cr.Vt[2] + cr.al * ((double)vz[k] - cr.Vn[2]));
                        const double x = vx[k], y = vy[k], z = vz[k];
                        real[0] += x;
                        real[1] += y;
                        real[2] += z;
                        real[3] += x * x + y * y + z * z;
                    }
                }
                const double t = block_sum_scatter<4>(real, red);
                if (a.debt) store_debt_lane(a.debt + (int64_t)cell * 4, cr, t);
            }
        }
    }

    // null collisions: about 1% of the particles are candidates, so each lane
    // takes its candidates one at a time (selected out of its register slots)
    // instead of branching per slot, which would run the scattering for every
    // slot holding a candidate in any lane of the wave
    if constexpr (MCC) {
        uint32_t left = cand;
        while (__ballot(left != 0u) != 0ull) {
            if (left) {
                const int kk = __builtin_ctz(left);
                left &= left - 1u;
                R x = vx[0], y = vy[0], z = vz[0];
#pragma unroll
                for (int k = 1; k < K; ++k)
                    if (kk == k) {
                        x = vx[k];
                        y = vy[k];
                        z = vz[k];
                    }
                mcc_scatter<R>(x, y, z, pid_c[threadIdx.x + kk * T], a.seed, step, a.mass_ratio);
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (kk == k) {
                        vx[k] = x;
                        vy[k] = y;
                        vz[k] = z;
                    }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = threadIdx.x + k * T;
        if (i < n) {
            vx_g[i] = vx[k];
            vy_g[i] = vy[k];
            vz_g[i] = vz[k];
        }
    }
    if constexpr (MOM) cell_moments_out<R, T, K>(a.moments + (int64_t)cell * 14, vx, vy, vz, n, red);
    // every thread leaves the pass together: the caller's loop starts with a
    // thread-0 work fetch, and a thread-0 block just before it must not be
    // merged with it or moved out of the loop
    __syncthreads();
}

template <typename R, int T, int K, int F>
__global__ __launch_bounds__(T) void k_collide(CollideArgs a, const int32_t *__restrict__ list,
                                               int cls)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[16 * (T / PIC_WAVE)];
    __shared__ double s_before[4];
    __shared__ uint32_t wtot[T / PIC_WAVE];
    __shared__ int s_item;
    if (gated_off(a)) return;
    const uint32_t count = a.dflags->count[cls];
    if (blockIdx.x >= count) return;   // no work for this workgroup (nor a queue atomic)
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(&a.dflags->head[cls], 1u);
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item >= (int)count) break;
        cell_pass<R, T, K, F>(a, list[item], smem, red, wtot, s_before);
    }
}

// ------------------------------------------------------------ lean pass
// The binary32 pass of the plain step (optionally with the fused null
// collisions) for cells of up to T*K members, written for few VALU
// instructions and few LDS operations per member:
//   * bucket counters are whole words (no 16-bit packing), nb = 2^bits >= n
//     buckets, so a bucket holds 0.5..1 members on average;
//   * after the scan only members that share their bucket write their key
//     and index to LDS, and only they compare keys to rank themselves
//     (about half the members are alone in their bucket);
//   * the first member of each pair draws its Box-Muller deviate before the
//     exchange, so a record is 16 bytes (velocity and one word) and a cell of
//     up to lean_positions(T*K) members exchanges in one round;
//   * pair threads write both new velocities back in place; members read
//     their record.
// The pairs, the rotation (ta_half_z) and the null collisions are those of
// cell_pass, so the two give identical velocities.
// Workgroup barrier for LDS traffic only: waits for this wave's LDS
// operations, not for its global loads and stores (a __syncthreads would make
// every barrier wait for the velocity loads in flight and the stores of the
// previous cell).  The memory clobber keeps the compiler from moving memory
// accesses across it.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Inclusive scan of one word per lane over the wave with DPP: shifts by 1, 2,
// 4, 8 inside each 16-lane row, then the last lane of row 0 (2) added to row
// 1 (3) and the last lane of row 1 added to rows 2 and 3.
__device__ __forceinline__ uint32_t wave_incl_scan_dpp(uint32_t x)
{
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);   // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);   // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);   // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);   // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);   // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);   // row_bcast:31
    return x;
}

// Exclusive scan in place of the nb (a power of two) bucket counters, with
// cnt[nb] = total.  Thread t takes the contiguous run of per = nb / T
// counters starting at t per (one counter, or none, when nb < T): it sums
// them, the run totals are scanned across the wave (DPP) and the waves'
// totals added in order, then it writes its run's starts.  Contains the
// barriers.
template <int T, int PERMAX>
__device__ __forceinline__ void lds_excl_scan_runs(uint32_t *cnt, uint32_t nb, uint32_t *wtot)
{
    constexpr int NW = T / PIC_WAVE;
    const uint32_t lane = threadIdx.x & (PIC_WAVE - 1), wid = threadIdx.x / PIC_WAVE;
    const uint32_t per = nb >= (uint32_t)T ? nb / (uint32_t)T : (threadIdx.x < nb ? 1u : 0u);
    uint32_t *run = cnt + threadIdx.x * per;
    // the run is read twice (its sum, then its starts): no registers held
    // across the barrier
    uint32_t s = 0;
    if (PERMAX >= 4 && per >= 4u) {
#pragma unroll
        for (int c = 0; c < PERMAX; c += 4)
            if ((uint32_t)c < per) {
                const uint4 q = *(const uint4 *)(run + c);
                s += (q.x + q.y) + (q.z + q.w);
            }
    } else {
#pragma unroll
        for (int c = 0; c < (PERMAX < 4 ? PERMAX : 4); ++c)
            if ((uint32_t)c < per) s += run[c];
    }
    const uint32_t inc = wave_incl_scan_dpp(s);
    if (lane == PIC_WAVE - 1) wtot[wid] = inc;
    lds_barrier();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const uint32_t t = wtot[w];
        off += (uint32_t)w < wid ? t : 0u;
        tot += t;
    }
    uint32_t r = off + inc - s;
    if (PERMAX >= 4 && per >= 4u) {
#pragma unroll
        for (int c = 0; c < PERMAX; c += 4)
            if ((uint32_t)c < per) {
                const uint4 x = *(const uint4 *)(run + c);
                uint4 q;
                q.x = r;
                q.y = q.x + x.x;
                q.z = q.y + x.y;
                q.w = q.z + x.z;
                r = q.w + x.w;
                *(uint4 *)(run + c) = q;
            }
    } else {
#pragma unroll
        for (int c = 0; c < (PERMAX < 4 ? PERMAX : 4); ++c)
            if ((uint32_t)c < per) {
                const uint32_t x = run[c];
                run[c] = r;
                r += x;
            }
    }
    if (threadIdx.x == 0) cnt[nb] = tot;
    lds_barrier();
}

template <int T, int K>
struct LeanGeom {
    static constexpr int CAP = T * K;
    static constexpr int NBMAX = (int)next_pow2((uint32_t)CAP);
    static constexpr int PERMAX = NBMAX >= T ? NBMAX / T : 1;   // counters per thread
    static constexpr size_t CNT_WORDS = (size_t)NBMAX + 4;      // counters, starts, end
    static constexpr size_t SORT_BYTES = CNT_WORDS * 4 + ((size_t)CAP + 4) * 4 + (size_t)CAP * 2;
};

// Dynamic LDS the lean pass may use (its static part is below 512 bytes).
constexpr size_t LEAN_LDS_LIMIT = 160 * 1024 - 512;

// Positions exchanged per round: the whole cell when its records fit.
__host__ __device__ constexpr uint32_t lean_positions(int cap)
{
    const size_t want = ((size_t)cap + 1) & ~(size_t)1;
    const size_t lim = (LEAN_LDS_LIMIT / sizeof(Rec<float>)) & ~(size_t)63;
    return (uint32_t)(want < lim ? want : lim);
}

template <int T, int K>
__host__ __device__ constexpr size_t lean_lds_bytes()
{
    const size_t ex = (size_t)lean_positions(T * K) * sizeof(Rec<float>);
    const size_t s = LeanGeom<T, K>::SORT_BYTES;
    return s > ex ? s : ex;
}

// One exchange round over the sorted positions [base, base + P): members post
// (velocity, word) at their position (the unpaired last one too), one thread
// per pair rotates, null-collision candidates scatter their records, members
// read their record back.  Contains the barriers.
template <int T, int K, bool MCC>
__device__ __forceinline__ void lean_round(uint32_t base, uint32_t P, uint32_t np2, int n, float C,
                                           Rec<float> *rec, float (&vx)[K], float (&vy)[K],
                                           float (&vz)[K], const uint32_t (&w2)[K],
                                           const uint32_t (&w3)[K], const uint32_t (&pos)[K],
                                           uint32_t &cand, int kf, uint32_t cpid,
                                           const uint32_t *pid_c, const CollideArgs &a,
                                           uint32_t step)
{
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = threadIdx.x + k * T;
        const uint32_t q = pos[k] - base;
        if (i < n && q < P) {
            // first members carry their deviate, second ones word 2
            const float z = ta_z(w2[k], w3[k]);
            Rec<float> e;
            e.x = vx[k];
            e.y = vy[k];
            e.z = vz[k];
            e.w2 = (pos[k] & 1u) ? w2[k] : __float_as_uint(z);
            rec[q] = e;
        }
    }
    lds_barrier();
    const uint32_t m = min(P, np2 - base) / 2;
    for (uint32_t j = threadIdx.x; j < m; j += T) {
        Rec<float> A = rec[2 * j], B = rec[2 * j + 1];
        float hx, hy, hz;
        ta_half_z(A.x - B.x, A.y - B.y, A.z - B.z, C, __uint_as_float(A.w2), B.w2, hx, hy, hz);
        A.x += hx;
        A.y += hy;
        A.z += hz;
        B.x -= hx;
        B.y -= hy;
        B.z -= hz;
        rec[2 * j] = A;
        rec[2 * j + 1] = B;
    }
    lds_barrier();
    // null collisions of this round's candidates, on their own records (each
    // record is read back by its member's thread only, so no barrier), one
    // candidate at a time per lane; the pid of the thread's first candidate
    // (member kf) was kept from the sort
    if constexpr (MCC) {
        uint32_t left = cand, later = 0;
        while (__ballot(left != 0u) != 0ull) {
            if (left) {
                const int kk = __builtin_ctz(left);
                left &= left - 1u;
                uint32_t pk = pos[0];
#pragma unroll
                for (int k = 1; k < K; ++k)
                    if (kk == k) pk = pos[k];
                const uint32_t q = pk - base;
                if (q < P) {
                    uint32_t id = cpid;
                    if (kk != kf) {
                        // a later candidate (rare): its pid from memory, waited
                        // for here, so that the common path does not wait for
                        // the next cell's lines requested above
                        id = pid_c[threadIdx.x + kk * T];
                        asm volatile("" ::"v"(id));
                    }
                    Rec<float> e = rec[q];
                    mcc_scatter<float>(e.x, e.y, e.z, id, a.seed, step, a.mass_ratio);
                    rec[q] = e;
                } else {
                    later |= 1u << kk;
                }
            }
        }
        cand = later;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = threadIdx.x + k * T;
        const uint32_t q = pos[k] - base;
        if (i < n && q < P) {
            const Rec<float> e = rec[q];
            vx[k] = e.x;
            vy[k] = e.y;
            vz[k] = e.z;
        }
    }
}

// Element i of a cell's array as a uniform base plus a 32-bit byte offset
// (the scalar-base form of the global load and store): no 64-bit
// per-member address is formed or kept live.
template <typename X>
__device__ __forceinline__ X ld_at(const X *base, uint32_t i)
{
    return *(const X *)((const char *)base + (size_t)(i * (uint32_t)sizeof(X)));
}
template <typename X>
__device__ __forceinline__ void st_at(X *base, uint32_t i, X x)
{
    *(X *)((char *)base + (size_t)(i * (uint32_t)sizeof(X))) = x;
}

// s_waitcnt operand that waits for vector memory only: vmcnt (bits 3:0 and
// 15:14) 0, expcnt (6:4) and lgkmcnt (11:8) at their maxima.
constexpr int WAIT_VMCNT0 = 0x0F70;

// The member count as a value the compiler cannot see through: each phase
// tests its members against its own copy, so the per-member masks are not
// kept live (in scalar registers) from one phase to the next.
__device__ __forceinline__ int opaque(int n)
{
    asm volatile("" : "+s"(n));
    return n;
}

// Counting sort of a cell's members by (key, pid) in LDS, shared by the lean
// passes (n >= 2): one Philox call per member (key, words 2 and 3, the
// null-collision candidate bit; cpid: the pid of the thread's first
// candidate), bucket counts (at least one bucket per
// member), scan, placement, rank inside the buckets.  On entry pos[k] holds
// member k's pid, on return its position in the cell's sorted order.
// Contains the barriers; the sort's memory is free after a further barrier.
template <int T, int K, bool MCC, bool CLEAR2 = false>
__device__ __forceinline__ void lean_sort(const CollideArgs &a, int n, uint32_t step,
                                          const uint32_t *pid_c, unsigned char *smem, uint32_t *wtot,
                                          uint32_t (&w2)[K], uint32_t (&w3)[K], uint32_t (&key)[K],
                                          uint32_t (&pos)[K], uint32_t &cand, uint32_t &cpid)
{
    typedef LeanGeom<T, K> G;
    const uint32_t bits = sort_bits(n);
    const uint32_t nb = 1u << bits;
    const uint32_t per = nb >= (uint32_t)T ? nb / (uint32_t)T : 1u;
    uint32_t *cnt = (uint32_t *)smem;
    uint32_t *sk = cnt + G::CNT_WORDS;              // keys in sorted-slot order
    uint16_t *lst = (uint16_t *)(sk + G::CAP + 4);  // ... and their index in the cell
    // counters cleared two at a time (8-byte writes) in the binary32 pass
    // (the binary64 pass measured slower with them)
    if (CLEAR2 && G::PERMAX >= 2 && per >= 2u) {
#pragma unroll
        for (int q = 0; q < G::PERMAX / 2; ++q)
            if ((uint32_t)q < per / 2u) *(uint2 *)(cnt + 2 * (threadIdx.x + q * T)) = make_uint2(0u, 0u);
    } else {
#pragma unroll
        for (int q = 0; q < G::PERMAX; ++q)
            if ((uint32_t)q < per && threadIdx.x + q * T < nb) cnt[threadIdx.x + q * T] = 0u;
    }
    lds_barrier();
    // one Philox call per particle; count its key's bucket
    const int n1 = opaque(n);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = threadIdx.x + k * T;
        if (i < n1) {
            const W4 w = draw4(a.seed, pos[k], step, 0u, 0u);
            key[k] = w.x;
            w2[k] = w.z;
            w3[k] = w.w;
            if (MCC && (uint64_t)w.y < a.mcc_thr) {
                if (!cand) cpid = pos[k];
                cand |= 1u << k;
            }
            const uint32_t b = w.x >> (32u - bits);
            pos[k] = atomicAdd(&cnt[b], 1u);   // arrival rank in the bucket
        }
    }
    lds_barrier();
    // bucket starts (cnt[nb] = n)
    lds_excl_scan_runs<T, G::PERMAX>(cnt, nb, wtot);
    // slot = bucket start + arrival.  Every member posts its key at its slot
    // (the three slots past the last hold the largest key), members sharing
    // their bucket also their index; pos[k] becomes the bucket's start with
    // its size (15: 15 or more) in the top four bits.
    const int n2 = opaque(n);
    if (threadIdx.x < 3) sk[n2 + threadIdx.x] = 0xffffffffu;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = threadIdx.x + k * T;
        if (i < n2) {
            const uint32_t b = key[k] >> (32u - bits);
            const uint32_t st = cnt[b], size = cnt[b + 1] - st;
            const uint32_t slot = st + pos[k];
            sk[slot] = key[k];
            if (size > 1u) lst[slot] = (uint16_t)i;
            pos[k] = st | (min(size, 15u) << 28);
        }
    }
    lds_barrier();
    // rank by (key, pid) inside the bucket: the keys below this one among
    // the four slots from the bucket's start (slots of later buckets hold
    // larger keys) and the rest of the bucket
    const int n3 = opaque(n);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = threadIdx.x + k * T;
        if (i < n3) {
            const uint32_t st = pos[k] & 0x0fffffffu;
            uint32_t size = pos[k] >> 28;
            uint32_t r = 0, e = 0;
            uint32_t kj[4];
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j) kj[j] = sk[st + j];
            // one wait for the four reads
            asm volatile("" ::"v"(kj[0]), "v"(kj[1]), "v"(kj[2]), "v"(kj[3]));
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j) {
                r += kj[j] < key[k] ? 1u : 0u;
                e += kj[j] == key[k] ? 1u : 0u;
            }
            if (size > 4u) {
                if (size == 15u) size = cnt[(key[k] >> (32u - bits)) + 1u] - st;
                for (uint32_t j = st + 4u; j < st + size; ++j) {
                    const uint32_t kj = sk[j];
                    r += kj < key[k] ? 1u : 0u;
                    e += kj == key[k] ? 1u : 0u;
                }
            }
            if (e > 1u && size > 1u) {
                // equal keys (rare): the smaller pid comes first
                const uint32_t pi = pid_c[i];
                for (uint32_t j = st; j < st + size; ++j)
                    if (sk[j] == key[k] && pid_c[lst[j]] < pi) ++r;
            }
            pos[k] = st + r;
        }
    }
}

// The next cell's lines of pid and v are requested while this cell is still
// being worked on, so that its loads find them in the caches (the last-level
// cache holds every workgroup's next cell).  The loads go to LDS (a 256-byte
// sink that nothing reads): they write no register, so nothing waits for them
// before the next cell's own loads.
struct LeanNext {
    int *slot;                 // LDS word receiving the next work item
    unsigned *head;            // the queue's counter
    const int32_t *list;
    uint32_t count;
    float *sink;               // 64 words of LDS
};

template <int T>
__device__ __forceinline__ void prefetch_cell(const CollideArgs &a, int cell, float *sink)
{
    const int lo = a.cell_start[cell];
    const int n = a.cell_start[cell + 1] - lo;
    if (n <= 0) return;
    // 128-byte lines of each of the four arrays (one more for a start
    // inside a line); one dword per line
    const uint32_t lines = ((uint32_t)n + 31u) / 32u + 1u;
    for (uint32_t t = threadIdx.x; t < 4u * lines; t += T) {
        const uint32_t arr = t / lines, l = t - arr * lines;
        const uint32_t idx = (uint32_t)lo + min(l * 32u, (uint32_t)n - 1u);
        const float *p = arr == 0 ? (const float *)(a.pid + idx)
                                  : (const float *)a.v + (size_t)(arr - 1u) * (size_t)a.n + idx;
        __builtin_amdgcn_global_load_lds((const void *)p, (__attribute__((address_space(3))) void *)sink,
                                         4, 0, 0);
    }
}

// With nx, the pass also takes the next work item from the queue and
// returns it (every thread reads it after a barrier that follows its write
// and precedes the pass's end, so the next pass may overwrite the slot);
// without, it returns 0.
template <int T, int K, bool MCC>
__device__ __forceinline__ int lean_pass(const CollideArgs &a, int cell, unsigned char *smem, uint32_t *wtot,
                                         const LeanNext *nx = nullptr)
{
    typedef LeanGeom<T, K> G;
    constexpr uint32_t P = lean_positions(G::CAP);
    const int lo = a.cell_start[cell];
    const int n = a.cell_start[cell + 1] - lo;
    const uint32_t step = (uint32_t)read_step(a);
    float *vx_g = (float *)a.v + lo;
    float *vy_g = (float *)a.v + a.n + lo;
    float *vz_g = (float *)a.v + 2 * a.n + lo;
    const uint32_t *pid_c = a.pid + lo;

    float vx[K], vy[K], vz[K];
    uint32_t w2[K], w3[K], key[K], pos[K];
    uint32_t cand = 0;

    int next = 0;
    if (n == 0) {
        if (nx && threadIdx.x == 0) *nx->slot = (int)atomicAdd(nx->head, 1u);
        lds_barrier();   // leave together (see the end of the pass)
        if (nx) next = *nx->slot;
        lds_barrier();
        return next;
    }
    // every load of the thread is in flight before the first is used, the
    // ids first (the Philox calls wait for them only).  Members past the end
    // load the last one instead (ignored): with no branch around the loads the
    // compiler waits for each load by count instead of for all of them.
    {
        uint32_t ic[K];
#pragma unroll
        for (int k = 0; k < K; ++k) ic[k] = (uint32_t)min((int)threadIdx.x + k * T, n - 1);
#pragma unroll
        for (int k = 0; k < K; ++k) pos[k] = ld_at(pid_c, ic[k]);
        asm volatile("" ::: "memory");   // keep the id loads ahead of the velocity loads
#pragma unroll
        for (int k = 0; k < K; ++k) {
            vx[k] = ld_at((const float *)vx_g, ic[k]);
            vy[k] = ld_at((const float *)vy_g, ic[k]);
            vz[k] = ld_at((const float *)vz_g, ic[k]);
        }
    }
    // the next work item (issued behind this cell's loads, so waiting for it
    // costs nothing extra); read after a barrier below
    if (nx && threadIdx.x == 0) *nx->slot = (int)atomicAdd(nx->head, 1u);
    if (n >= 2) {
        uint32_t cpid = 0;
        lean_sort<T, K, MCC, true>(a, n, step, pid_c, smem, wtot, w2, w3, key, pos, cand, cpid);
        lds_barrier();   // the sort's memory becomes the exchange records

        const float C = (float)cell_C(a, cell);
        // last global loads before the exchange: a later wait for a load (the
        // density above) would wait for these too, so C is complete first
        if (nx) {
            asm volatile("" ::"v"(C));
            const uint32_t nxt = (uint32_t)*nx->slot;
            if (nxt < nx->count) prefetch_cell<T>(a, nx->list[nxt], nx->sink);
        }
        const uint32_t np2 = (uint32_t)n & ~1u;     // positions with a partner
        Rec<float> *rec = (Rec<float> *)smem;
        const int kf = cand ? __builtin_ctz(cand) : K;
        for (uint32_t base = 0; base < (uint32_t)n; base += P) {
            if (base) lds_barrier();
            lean_round<T, K, MCC>(base, P, np2, opaque(n), C, rec, vx, vy, vz, w2, w3, pos, cand,
                                  kf, cpid, pid_c, a, step);
        }
    } else if (MCC) {
        const W4 w = draw4(a.seed, pos[0], step, 0u, 0u);
        if (threadIdx.x == 0 && (uint64_t)w.y < a.mcc_thr) cand = 1u;
    }

    // null collision of a lone member (n = 1: thread 0's member 0, whose pid
    // is in pos[0]; the exchange rounds took every candidate of a larger cell)
    if (MCC && cand) mcc_scatter<float>(vx[0], vy[0], vz[0], pos[0], a.seed, step, a.mass_ratio);
    // one wait for every load still outstanding (the next cell's lines,
    // requested long before) ahead of the stores: the compiler would otherwise
    // wait before each member's stores, and each wait drains the stores
    // before it too
    if (nx) __builtin_amdgcn_s_waitcnt(WAIT_VMCNT0);
    const int n3 = opaque(n);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = threadIdx.x + k * T;
        if (i < n3) {
            vx_g[i] = vx[k];
            vy_g[i] = vy[k];
            vz_g[i] = vz[k];
        }
    }
    // the next item: written by thread 0 before at least one barrier of
    // this pass when n >= 2 (else one more barrier), read by everyone before
    // the last one (the next pass writes it only after that)
    if (nx) {
        if (n < 2) lds_barrier();
        next = *nx->slot;
    }
    // the next cell reuses the LDS; the stores stay in flight into it
    lds_barrier();
    return next;
}

template <int T, int K, bool MCC>
__global__ __launch_bounds__(T) void k_collide_lean(CollideArgs a, const int32_t *__restrict__ list,
                                                    int cls)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t wtot[T / PIC_WAVE];
    __shared__ int s_item, s_next;
    __shared__ float sink[PIC_WAVE];
    if (gated_off(a)) return;
    const uint32_t count = a.dflags->count[cls];
    if (blockIdx.x >= count) return;   // no work for this workgroup (nor a queue atomic)
    if (threadIdx.x == 0) s_item = (int)atomicAdd(&a.dflags->head[cls], 1u);
    lds_barrier();
    int item = s_item;
    const LeanNext nx{&s_next, &a.dflags->head[cls], list, count, sink};
    while (item < (int)count) item = lean_pass<T, K, MCC>(a, list[item], smem, wtot, &nx);
}

// ------------------------------------------------------------ lean pass, binary64
// The plain binary64 step (optionally with the fused null collisions) for
// cells of up to T*K members on one workgroup: the lean pass's sort, then the
// exchange in rounds of Lean64Geom::P sorted positions (two for a
// 10,000-member cell): the round's members load their velocity and post it
// with their words 2 and 3 at their position, one thread per pair computes
// the binary64 half change (ta_half, the oracle's order of operations) and
// writes both members back, the round's members read their record, scatter
// if they are null-collision candidates, and store it.  No velocity is held
// in registers across a round, which leaves the register file to the
// binary64 rotation.  The pairs, the rotation and the null collisions are
// those of cell_pass.


template <int T, int K>
struct Lean64Geom {
    static constexpr int CAP = T * K;
    static constexpr uint32_t P = (uint32_t)((LEAN_LDS_LIMIT / sizeof(Rec<double>)) & ~(size_t)63);
    static constexpr size_t BYTES = (size_t)P * sizeof(Rec<double>);
};

template <int T, int K>
__host__ __device__ constexpr size_t lean64_lds_bytes()
{
    typedef Lean64Geom<T, K> G;
    const size_t s = LeanGeom<T, K>::SORT_BYTES;
    return s > G::BYTES ? s : G::BYTES;
}

template <int T, int K, bool MCC>
__device__ __forceinline__ void lean64_pass(const CollideArgs &a, int cell, unsigned char *smem,
                                            uint32_t *wtot, float *sink)
{
    typedef Lean64Geom<T, K> G;
    constexpr uint32_t P = G::P;
    const int lo = a.cell_start[cell];
    const int n = a.cell_start[cell + 1] - lo;
    const uint32_t step = (uint32_t)read_step(a);
    double *vx_g = (double *)a.v + lo;
    double *vy_g = (double *)a.v + a.n + lo;
    double *vz_g = (double *)a.v + 2 * a.n + lo;
    const uint32_t *pid_c = a.pid + lo;

    uint32_t pos[K];
    uint32_t cand = 0;
    if (n == 0) {
        lds_barrier();
        return;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) pos[k] = pid_c[min((int)threadIdx.x + k * T, n - 1)];
    // the cell's velocity lines are requested now (into an LDS sink, no
    // register written), so that the rounds' loads find them cached
    {
        const uint32_t lines = ((uint32_t)n + 15u) / 16u + 1u;   // 128-byte lines of doubles
        for (uint32_t t = threadIdx.x; t < 3u * lines; t += T) {
            const uint32_t arr = t / lines, l = t - arr * lines;
            const double *p = (const double *)a.v + (size_t)arr * (size_t)a.n + (uint32_t)lo +
                              min(l * 16u, (uint32_t)n - 1u);
            __builtin_amdgcn_global_load_lds((const void *)p, (__attribute__((address_space(3))) void *)sink,
                                             4, 0, 0);
        }
    }
    uint32_t np2 = 0;
    if (n >= 2) {
        uint32_t w2[K], w3[K];
        {
            uint32_t key[K], cpid = 0;
            lean_sort<T, K, MCC>(a, n, step, pid_c, smem, wtot, w2, w3, key, pos, cand, cpid);
        }
        lds_barrier();   // the sort's memory becomes the records
        Rec<double> *rec = (Rec<double> *)smem;
        const double C = cell_C(a, cell);
        np2 = (uint32_t)n & ~1u;
        for (uint32_t base = 0; base < np2; base += P) {
            if (base) lds_barrier();
            // the thread index as a per-round value the compiler cannot hoist:
            // each round recomputes its members' offsets instead of keeping
            // them all live from the kernel's start
            uint32_t tid = threadIdx.x;
            asm volatile("" : "+v"(tid));
            {
                // loads in two halves, each posted before the next is loaded
                // (all ten members' velocities at once would not fit beside
                // the rotation's constants)
                constexpr int H = (K + 1) / 2;
#pragma unroll
                for (int h = 0; h < K; h += H) {
                    const int n4 = opaque(n);
                    double x[H], y[H], z[H];
#pragma unroll
                    for (int kk = 0; kk < H; ++kk) {
                        const int k = h + kk;
                        if (k < K) {
                            const int i = (int)tid + k * T;
                            const uint32_t q = pos[k] - base;
                            if (i < n4 && q < P && pos[k] < np2) {
                                x[kk] = ld_at(vx_g, (uint32_t)i);
                                y[kk] = ld_at(vy_g, (uint32_t)i);
                                z[kk] = ld_at(vz_g, (uint32_t)i);
                            }
                        }
                    }
#pragma unroll
                    for (int kk = 0; kk < H; ++kk) {
                        const int k = h + kk;
                        if (k < K) {
                            const int i = (int)tid + k * T;
                            const uint32_t q = pos[k] - base;
                            if (i < n4 && q < P && pos[k] < np2) {
                                Rec<double> e;
                                e.x = x[kk];
                                e.y = y[kk];
                                e.z = z[kk];
                                e.w2 = w2[k];
                                e.pad = w3[k];
                                rec[q] = e;
                            }
                        }
                    }
                }
            }
            lds_barrier();
            const uint32_t m = min(P, np2 - base) / 2;
            for (uint32_t j = threadIdx.x; j < m; j += T) {
                Rec<double> A = rec[2 * j], B = rec[2 * j + 1];
                double hx, hy, hz;
                ta_half(A.x - B.x, A.y - B.y, A.z - B.z, C, A.w2, A.pad, B.w2, hx, hy, hz);
                A.x += hx;
                A.y += hy;
                A.z += hz;
                B.x -= hx;
                B.y -= hy;
                B.z -= hz;
                rec[2 * j] = A;
                rec[2 * j + 1] = B;
            }
            lds_barrier();
            // the round's members store their record (null-collision
            // candidates after their scattering, one at a time per lane); the
            // members' offsets and tests are recomputed, not kept from the posts
            const int n5 = opaque(n);
            asm volatile("" : "+v"(tid));
            uint32_t base5 = base;
            asm volatile("" : "+s"(base5));
            uint32_t left = 0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int i = (int)tid + k * T;
                const uint32_t q = pos[k] - base5;
                if (i < n5 && q < P && pos[k] < np2) {
                    if (MCC && ((cand >> k) & 1u)) {
                        left |= 1u << k;
                    } else {
                        const Rec<double> e = rec[q];
                        st_at(vx_g, (uint32_t)i, e.x);
                        st_at(vy_g, (uint32_t)i, e.y);
                        st_at(vz_g, (uint32_t)i, e.z);
                    }
                }
            }
            if constexpr (MCC) {
                while (__ballot(left != 0u) != 0ull) {
                    if (left) {
                        const int kk = __builtin_ctz(left);
                        left &= left - 1u;
                        uint32_t pk = pos[0];
#pragma unroll
                        for (int k = 1; k < K; ++k)
                            if (kk == k) pk = pos[k];
                        const int i = (int)tid + kk * T;
                        const Rec<double> e = rec[pk - base5];
                        double x = e.x, y = e.y, z = e.z;
                        mcc_scatter<double>(x, y, z, pid_c[i], a.seed, step, a.mass_ratio);
                        st_at(vx_g, (uint32_t)i, x);
                        st_at(vy_g, (uint32_t)i, y);
                        st_at(vz_g, (uint32_t)i, z);
                    }
                }
            }
        }
    } else if (MCC) {
        const W4 w = draw4(a.seed, pos[0], step, 0u, 0u);
        if (threadIdx.x == 0 && (uint64_t)w.y < a.mcc_thr) cand = 1u;
    }
    // the member without a partner (odd n) keeps its velocity, apart from
    // its null collision
    if constexpr (MCC) {
        uint32_t left = 0;
        const int n6 = opaque(n);
#pragma unroll
        for (int k = 0; k < K; ++k)
            if ((int)threadIdx.x + k * T < n6 && ((cand >> k) & 1u) && (n < 2 || pos[k] >= np2))
                left |= 1u << k;
        if (left) {
            const int kk = __builtin_ctz(left);   // at most one such member per cell
            const int i = threadIdx.x + kk * T;
            double x = ld_at(vx_g, (uint32_t)i), y = ld_at(vy_g, (uint32_t)i), z = ld_at(vz_g, (uint32_t)i);
            mcc_scatter<double>(x, y, z, pid_c[i], a.seed, step, a.mass_ratio);
            st_at(vx_g, (uint32_t)i, x);
            st_at(vy_g, (uint32_t)i, y);
            st_at(vz_g, (uint32_t)i, z);
        }
    }
    lds_barrier();   // the next cell reuses the LDS
}

template <int T, int K, bool MCC>
__global__ __launch_bounds__(T) void k_collide_lean64(CollideArgs a, const int32_t *__restrict__ list,
                                                      int cls)
{
    // one cell per workgroup (not persistent: a loop over cells would let
    // the compiler hoist the rotation's constants and the members' offsets
    // to the kernel's start and keep them live through every cell)
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t wtot[T / PIC_WAVE];
    __shared__ float sink[PIC_WAVE];
    if (gated_off(a)) return;
    if (blockIdx.x >= a.dflags->count[cls]) return;
    lean64_pass<T, K, MCC>(a, list[blockIdx.x], smem, wtot, sink);
}

// ------------------------------------------------------------ huge cells
// One workgroup per cell; per-particle state in global scratch indexed by the
// particle's slot, so scratch regions of different cells never overlap.
template <typename R, bool PAIRS>
__global__ __launch_bounds__(1024) void k_collide_huge(CollideArgs a, const int32_t *__restrict__ list,
                                                       int cls, HugeScratch hs,
                                                       const uint8_t *__restrict__ only)
{
    __shared__ double red[16 * 16];
    __shared__ uint32_t wtot[16];
    __shared__ int s_item;
    if (gated_off(a)) return;
    if (only && !a.dflags->seg_fallback) return;   // every cell went the segmented way
    const uint32_t count = a.dflags->count[cls];
    if (blockIdx.x >= count) return;   // no work for this workgroup (nor a queue atomic)
    const int T = blockDim.x;
    R *vx_g = (R *)a.v;
    R *vy_g = vx_g + a.n;
    R *vz_g = vy_g + a.n;
    Rec<R> *pb = (Rec<R> *)hs.pbuf;
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(&a.dflags->head[cls], 1u);
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item >= (int)count) break;
        if (only && !only[item]) continue;   // taken by the segmented path
        const int cell = list[item];
        const int lo = a.cell_start[cell];
        const int n = a.cell_start[cell + 1] - lo;
        const uint32_t step = (uint32_t)read_step(a);
        const bool coul = n >= 2;
        double before[4] = {0, 0, 0, 0};   // sum v, sum |v|^2
        for (int i = threadIdx.x; i < n; i += T) {
            const W4 w = draw4(a.seed, a.pid[lo + i], step, 0u, 0u);
            hs.keys[lo + i] = w.x;
            hs.w23[2 * (int64_t)(lo + i)] = w.z;
            hs.w23[2 * (int64_t)(lo + i) + 1] = w.w;
            hs.cand[lo + i] = (uint64_t)w.y < a.mcc_thr;
            if (!PAIRS && (a.flags & PIC_CONSERVE_FIX)) {
                const double x = vx_g[lo + i], y = vy_g[lo + i], z = vz_g[lo + i];
                before[0] += x;
                before[1] += y;
                before[2] += z;
                before[3] += x * x + y * y + z * z;
            }
        }
        __syncthreads();
        if (coul || PAIRS) gsort_positions(hs, a.pid, lo, n, wtot);
        if (PAIRS) {
            for (int i = threadIdx.x; i < n; i += T) a.sorted_out[lo + hs.pos[lo + i]] = lo + i;
            for (int i = threadIdx.x; i < n; i += T) {
                const uint32_t q = hs.pos[lo + i] ^ 1u;
                a.partner_out[lo + i] = (q < (uint32_t)n) ? lo + (int)hs.lst[lo + q] : -1;
            }
            __syncthreads();
            continue;
        }
        if (coul) {
            const R C = (R)cell_C(a, cell);
            Rec<R> *pc = pb + lo / 2 + (lo & 1);   // disjoint per cell
            for (int i = threadIdx.x; i < n; i += T) {
                const uint32_t p = hs.pos[lo + i];
                if (p & 1u) {
                    Rec<R> &e = pc[p >> 1];
                    e.x = vx_g[lo + i];
                    e.y = vy_g[lo + i];
                    e.z = vz_g[lo + i];
                    e.w2 = hs.w23[2 * (int64_t)(lo + i)];
                }
            }
            __syncthreads();
            // with the triplet, an odd cell's last three positions form it
            const uint32_t tstart = (a.variant == VAR_TRIPLET && (n & 1) && n >= 3) ? (uint32_t)n - 3u
                                                                                 : (uint32_t)n & ~1u;
            for (int i = threadIdx.x; i < n; i += T) {
                const uint32_t p = hs.pos[lo + i];
                if (!(p & 1u) && p + 1 < tstart) {
                    Rec<R> &e = pc[p >> 1];
                    R x = vx_g[lo + i], y = vy_g[lo + i], z = vz_g[lo + i];
                    R hx, hy, hz;
                    if (a.variant == VAR_NANBU) {
                        // the member in the lower storage slot is the operator's first
                        const uint32_t j = hs.lst[lo + p + 1];
                        const uint32_t own = hs.w23[2 * (int64_t)(lo + i)];
                        if ((uint32_t)i < j) {
                            nanbu_half<R>(x - e.x, y - e.y, z - e.z, C, own, e.w2, hx, hy, hz);
                        } else {
                            nanbu_half<R>(e.x - x, e.y - y, e.z - z, C, e.w2, own, hx, hy, hz);
                            hx = -hx;
                            hy = -hy;
                            hz = -hz;
                        }
                    } else {
                        ta_half(x - e.x, y - e.y, z - e.z, C, hs.w23[2 * (int64_t)(lo + i)],
                                hs.w23[2 * (int64_t)(lo + i) + 1], e.w2, hx, hy, hz);
                    }
                    bool ta = true, tb = true;
                    if (a.w) {
                        // the partner: the member at the next position
                        const R *wg = (const R *)a.w + lo;
                        const uint32_t j = hs.lst[lo + p + 1];
                        weight_rule<R>(wg[i], wg[j], hs.w23[2 * (int64_t)(lo + j) + 1], ta, tb);
                    }
                    if (ta) {
                        vx_g[lo + i] = x + hx;
                        vy_g[lo + i] = y + hy;
                        vz_g[lo + i] = z + hz;
                    }
                    // the second member subtracts what is left here
                    e.x = tb ? hx : (R)0;
                    e.y = tb ? hy : (R)0;
                    e.z = tb ? hz : (R)0;
                }
            }
            __syncthreads();
            for (int i = threadIdx.x; i < n; i += T) {
                const uint32_t p = hs.pos[lo + i];
                if ((p & 1u) && p < tstart) {
                    const Rec<R> &e = pc[p >> 1];
                    vx_g[lo + i] -= e.x;
                    vy_g[lo + i] -= e.y;
                    vz_g[lo + i] -= e.z;
                }
            }
            __syncthreads();
            if (tstart + 3 == (uint32_t)n && (n & 1) && threadIdx.x == 0) {
                // the triplet: one thread, members read through the sorted list
                int64_t sl[3];
                R x[3], y[3], z[3];
                uint32_t pd[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    sl[c] = lo + (int64_t)hs.lst[lo + tstart + c];
                    x[c] = vx_g[sl[c]];
                    y[c] = vy_g[sl[c]];
                    z[c] = vz_g[sl[c]];
                    pd[c] = a.pid[sl[c]];
                }
                const double dens = a.density ? a.density[cell] : 1.0;
                triplet_collide<R>(x, y, z, pd, (R)(8.0 * PI_D * dens * a.lnL * (0.5 * a.dt)), a.seed,
                                   step);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    vx_g[sl[c]] = x[c];
                    vy_g[sl[c]] = y[c];
                    vz_g[sl[c]] = z[c];
                }
            }
            __syncthreads();
            if (a.flags & PIC_CONSERVE_FIX) {
                double after[4] = {0, 0, 0, 0};
                for (int i = threadIdx.x; i < n; i += T) {
                    const double x = vx_g[lo + i], y = vy_g[lo + i], z = vz_g[lo + i];
                    after[0] += x;
                    after[1] += y;
                    after[2] += z;
                    after[3] += x * x + y * y + z * z;
                }
                block_sum<4>(before, red);
                block_sum<4>(after, red);
                const Correction cr = make_correction((double)n, before, after,
                                                      a.debt ? a.debt + (int64_t)cell * 4 : nullptr);
                if (cr.ok) {
                    double real[4] = {0, 0, 0, 0};
                    for (int i = threadIdx.x; i < n; i += T) {
                        const R x = (R)(cr.Vt[0] + cr.al * ((double)vx_g[lo + i] - cr.Vn[0]));
                        const R y = (R)(cr.Vt[1] + cr.al * ((double)vy_g[lo + i] - cr.Vn[1]));
                        const R z = (R)(cr.Vt[2] + cr.al * ((double)vz_g[lo + i] - cr.Vn[2]));
                        vx_g[lo + i] = x;
                        vy_g[lo + i] = y;
                        vz_g[lo + i] = z;
                        real[0] += (double)x;
                        real[1] += (double)y;
                        real[2] += (double)z;
                        real[3] += (double)x * x + (double)y * y + (double)z * z;
                    }
                    block_sum<4>(real, red);
                    if (a.debt && threadIdx.x == 0) store_debt(a.debt + (int64_t)cell * 4, cr, real);
                }
                __syncthreads();
            }
        }
        double m[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) m[q] = 0.0;
        for (int i = threadIdx.x; i < n; i += T) {
            R x = vx_g[lo + i], y = vy_g[lo + i], z = vz_g[lo + i];
            if (a.mcc_thr && hs.cand[lo + i]) {
                mcc_scatter<R>(x, y, z, a.pid[lo + i], a.seed, step, a.mass_ratio);
                vx_g[lo + i] = x;
                vy_g[lo + i] = y;
                vz_g[lo + i] = z;
            }
            if (a.flags & PIC_MOMENTS) moment_terms(m, x, y, z);
        }
        if (a.flags & PIC_MOMENTS) {
            const double t = block_sum_scatter<16>(m, red);
            if (threadIdx.x < 14) a.moments[(int64_t)cell * 14 + threadIdx.x] = t;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ segmented cells
// Cells beyond the largest LDS class with several workgroups each (see
// SegScratch): count members per segment, scan, copy members segment-major,
// sort and pair each segment in LDS, then the pairs across segment edges.
constexpr int SEG_CT = 256;   // threads of the counting and copying kernels
constexpr int SEG_U = 8;      // members per thread whose loads are in flight together

// Segment of a key among S equal key ranges, and the key's position inside
// its range scaled to 32 bits (order-preserving within the segment).
__device__ __forceinline__ uint32_t seg_of(uint32_t key, uint32_t S)
{
    return (uint32_t)(((uint64_t)key * S) >> 32);
}
__device__ __forceinline__ uint32_t seg_key(uint32_t key, uint32_t S)
{
    return (uint32_t)((uint64_t)key * S);
}

struct SegItem {
    int h, lo, b, e;
    uint32_t S;
};

// Work item -> its cell h of the list, the cell's first slot and the item's
// member range [b, e) inside the cell.
__device__ __forceinline__ SegItem seg_item(const CollideArgs &a, const SegScratch &ss,
                                            const int32_t *list, uint32_t item)
{
    SegItem it;
    it.h = ss.ch_owner[item];
    const int cell = list[it.h];
    it.lo = a.cell_start[cell];
    const int n = a.cell_start[cell + 1] - it.lo;
    it.b = (int)(item - (uint32_t)ss.hc_chunk[it.h]) * SEG_CHUNK;
    it.e = min(n, it.b + SEG_CHUNK);
    it.S = ss.hc_S[it.h];
    return it;
}

// Segment sizes: an LDS histogram per work item, then one global add per
// non-empty segment.
__global__ __launch_bounds__(SEG_CT) void k_seg_count(CollideArgs a, const int32_t *__restrict__ list,
                                                      SegScratch ss)
{
    __shared__ uint32_t hist[SEG_MAX];
    if (gated_off(a)) return;
    const uint32_t items = a.dflags->count[CHUNK_SLOT];
    const uint32_t step = (uint32_t)read_step(a);
    for (uint32_t item = blockIdx.x; item < items; item += gridDim.x) {
        const SegItem it = seg_item(a, ss, list, item);
        const uint32_t S = it.S;
        for (uint32_t q = threadIdx.x; q < S; q += SEG_CT) hist[q] = 0u;
        __syncthreads();
        // SEG_U members per thread per round, their pids loaded together
        for (int i0 = it.b + (int)threadIdx.x; i0 < it.e; i0 += SEG_U * SEG_CT) {
            uint32_t pv[SEG_U];
#pragma unroll
            for (int u = 0; u < SEG_U; ++u) {
                const int i = i0 + u * SEG_CT;
                if (i < it.e) pv[u] = a.pid[it.lo + i];
            }
#pragma unroll
            for (int u = 0; u < SEG_U; ++u) {
                const int i = i0 + u * SEG_CT;
                if (i < it.e) atomicAdd(&hist[seg_of(draw4(a.seed, pv[u], step, 0u, 0u).x, S)], 1u);
            }
        }
        __syncthreads();
        const int32_t sb = ss.hc_seg[it.h];
        for (uint32_t q = threadIdx.x; q < S; q += SEG_CT)
            if (hist[q]) atomicAdd(&ss.sg_cnt[sb + q], hist[q]);
        __syncthreads();
    }
}

// One workgroup: each segment's run in the scratch (exclusive scan of the
// sizes in table order) and the copy cursors; a cell with a segment beyond
// cap takes the one-workgroup path.
__global__ __launch_bounds__(1024) void k_seg_scan(CollideArgs a, SegScratch ss, uint32_t cap)
{
    __shared__ uint32_t wtot[16];
    __shared__ uint32_t s_tot;
    if (gated_off(a)) return;
    const uint32_t nseg = a.dflags->count[SEG_SLOT];
    uint32_t base = 0;
    for (uint32_t j0 = 0; j0 < nseg; j0 += 1024) {
        const uint32_t j = j0 + threadIdx.x;
        const uint32_t c = j < nseg ? ss.sg_cnt[j] : 0u;
        const uint32_t off = block_excl(c, wtot);
        if (j < nseg) {
            ss.sg_start[j] = base + off;
            ss.sg_cur[j] = base + off;
            if (c > cap) {
                ss.hc_fb[ss.sg_cell[j]] = 1;
                a.dflags->seg_fallback = 1;
            }
        }
        if (threadIdx.x == 1023) s_tot = off + c;
        __syncthreads();
        base += s_tot;
        __syncthreads();
    }
}

// Members to their segment's run: counts per segment in LDS, one global
// reservation per non-empty segment, then each member at its reservation
// plus its LDS arrival rank (the order inside a run is free: the segment
// pass sorts by key and pid).
template <typename R>
__global__ __launch_bounds__(SEG_CT) void k_seg_scatter(CollideArgs a, const int32_t *__restrict__ list,
                                                        SegScratch ss)
{
    __shared__ uint32_t hist[SEG_MAX];
    __shared__ uint32_t base[SEG_MAX];
    __shared__ uint16_t sof[SEG_CHUNK];
    if (gated_off(a)) return;
    const uint32_t items = a.dflags->count[CHUNK_SLOT];
    const uint32_t step = (uint32_t)read_step(a);
    const R *v = (const R *)a.v;
    R *mv = (R *)ss.m_v;
    for (uint32_t item = blockIdx.x; item < items; item += gridDim.x) {
        const SegItem it = seg_item(a, ss, list, item);
        if (ss.hc_fb[it.h]) continue;   // the same for the whole workgroup
        const uint32_t S = it.S;
        for (uint32_t q = threadIdx.x; q < S; q += SEG_CT) hist[q] = 0u;
        __syncthreads();
        for (int i0 = it.b + (int)threadIdx.x; i0 < it.e; i0 += SEG_U * SEG_CT) {
            uint32_t pv[SEG_U];
#pragma unroll
            for (int u = 0; u < SEG_U; ++u) {
                const int i = i0 + u * SEG_CT;
                if (i < it.e) pv[u] = a.pid[it.lo + i];
            }
#pragma unroll
            for (int u = 0; u < SEG_U; ++u) {
                const int i = i0 + u * SEG_CT;
                if (i < it.e) {
                    const uint32_t q = seg_of(draw4(a.seed, pv[u], step, 0u, 0u).x, S);
                    sof[i - it.b] = (uint16_t)q;
                    atomicAdd(&hist[q], 1u);
                }
            }
        }
        __syncthreads();
        const int32_t sb = ss.hc_seg[it.h];
        for (uint32_t q = threadIdx.x; q < S; q += SEG_CT) {
            base[q] = hist[q] ? atomicAdd(&ss.sg_cur[sb + q], hist[q]) : 0u;
            hist[q] = 0u;
        }
        __syncthreads();
        for (int i0 = it.b + (int)threadIdx.x; i0 < it.e; i0 += SEG_U * SEG_CT) {
            uint32_t pv[SEG_U];
            R x[SEG_U], y[SEG_U], z[SEG_U];
#pragma unroll
            for (int u = 0; u < SEG_U; ++u) {
                const int64_t g = (int64_t)it.lo + i0 + u * SEG_CT;
                if (i0 + u * SEG_CT < it.e) {
                    pv[u] = a.pid[g];
                    x[u] = v[g];
                    y[u] = v[a.n + g];
                    z[u] = v[2 * a.n + g];
                }
            }
#pragma unroll
            for (int u = 0; u < SEG_U; ++u) {
                const int i = i0 + u * SEG_CT;
                if (i < it.e) {
                    const uint32_t q = sof[i - it.b];
                    const uint32_t slot = base[q] + atomicAdd(&hist[q], 1u);
                    ss.m_orig[slot] = it.lo + i;
                    ss.m_pid[slot] = pv[u];
                    mv[slot] = x[u];
                    mv[ss.m_stride + slot] = y[u];
                    mv[2 * ss.m_stride + slot] = z[u];
                }
            }
        }
        __syncthreads();
    }
}

// One segment: the members of run [start, start + n) sort by key (by their
// position inside the segment's key range, scaled to 32 bits, whose top bits
// bucket them) and pid; local
// position q is position off + q of the cell.  The cell's pairs (2i, 2i + 1)
// inside the segment collide here as in the cell pass; a member whose
// partner lies in a neighbouring segment is recorded for k_seg_fixup and left
// unchanged (its null collision too).
template <typename R, int T, int K, int F>
__device__ __forceinline__ void seg_pass(const CollideArgs &a, const int32_t *list, const SegScratch &ss, int seg,
                         unsigned char *smem, uint32_t *wtot)
{
    constexpr bool MCC = (F & F_MCC) != 0;
    constexpr int CAP = T * K;
    const int h = ss.sg_cell[seg];
    const uint32_t n = ss.sg_cnt[seg];
    if (ss.hc_fb[h] || n == 0) {
        __syncthreads();
        return;
    }
    const int cell = list[h];
    const int lo_c = a.cell_start[cell];
    const uint32_t n_c = (uint32_t)(a.cell_start[cell + 1] - lo_c);
    const uint32_t start = ss.sg_start[seg];
    const uint32_t off = start - ss.sg_start[ss.hc_seg[h]];
    const uint32_t S = ss.hc_S[h];
    const uint32_t step = (uint32_t)read_step(a);
    const R *mx = (const R *)ss.m_v + start;
    const R *my = mx + ss.m_stride;
    const R *mz = my + ss.m_stride;
    const uint32_t *pid_s = ss.m_pid + start;
    const int32_t *orig = ss.m_orig + start;
    R *vx_g = (R *)a.v;
    R *vy_g = vx_g + a.n;
    R *vz_g = vy_g + a.n;
    const SortLDS<T, CAP> L(smem);

    R vx[K], vy[K], vz[K];
    uint32_t w2[K], w3[K], pos[K];
    uint32_t cand = 0;
    const uint32_t bits = sort_bits((int)n);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = threadIdx.x + k * T;
        if (i < (int)n) {
            pos[k] = pid_s[i];
            vx[k] = mx[i];
            vy[k] = my[i];
            vz[k] = mz[i];
        }
    }
    L.clear();
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = threadIdx.x + k * T;
        if (i < (int)n) {
            const W4 w = draw4(a.seed, pos[k], step, 0u, 0u);
            w2[k] = w.z;
            w3[k] = w.w;
            if (MCC && (uint64_t)w.y < a.mcc_thr) cand |= 1u << k;
            pos[k] = L.count(i, seg_key(w.x, S), bits);
        }
    }
    __syncthreads();
    rank_in_lds<T, K, CAP>(pos, (int)n, bits, L, pid_s, wtot);

    // local pairs cover positions [first, first + np2)
    const uint32_t first = off & 1u;
    const uint32_t np2 = (n - first) & ~1u;
    uint32_t edge = 0;   // bit k: the partner is in a neighbouring segment
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = threadIdx.x + k * T;
        if (i < (int)n) {
            if (first && pos[k] == 0u) {
                edge |= 1u << k;
                ss.bnd_head[seg] = (int32_t)(start + i);
            } else if (pos[k] == first + np2 && off + pos[k] + 1u < n_c) {
                edge |= 1u << k;
                ss.bnd_tail[seg] = (int32_t)(start + i);
            }
        }
    }
    {
        const R C = (R)cell_C(a, cell);
        constexpr uint32_t P = round_positions<R>(CAP);
        Rec<R> *rec = (Rec<R> *)smem;
        uint32_t *w3s = (uint32_t *)(rec + P);
        for (uint32_t base = 0; base < np2; base += P) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int i = threadIdx.x + k * T;
                const uint32_t pl = pos[k] - first;   // wraps for the lower edge member
                const uint32_t q = pl - base;
                if (i < (int)n && pl < np2 && q < P) {
                    Rec<R> e;
                    e.x = vx[k];
                    e.y = vy[k];
                    e.z = vz[k];
                    e.w2 = w2[k];
                    rec[q] = e;
                    if (!(q & 1u)) w3s[q >> 1] = w3[k];
                }
            }
            __syncthreads();
            const uint32_t m = min(P, np2 - base) / 2;
            for (uint32_t j = threadIdx.x; j < m; j += T) {
                Rec<R> A = rec[2 * j], B = rec[2 * j + 1];
                R hx, hy, hz;
                ta_half(A.x - B.x, A.y - B.y, A.z - B.z, C, A.w2, w3s[j], B.w2, hx, hy, hz);
                A.x += hx;
                A.y += hy;
                A.z += hz;
                B.x -= hx;
                B.y -= hy;
                B.z -= hz;
                rec[2 * j] = A;
                rec[2 * j + 1] = B;
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int i = threadIdx.x + k * T;
                const uint32_t pl = pos[k] - first;
                const uint32_t q = pl - base;
                if (i < (int)n && pl < np2 && q < P) {
                    const Rec<R> e = rec[q];
                    vx[k] = e.x;
                    vy[k] = e.y;
                    vz[k] = e.z;
                }
            }
            if (base + P < np2) __syncthreads();
        }
    }
    if constexpr (MCC) {
        uint32_t left = cand & ~edge;
        while (__ballot(left != 0u) != 0ull) {
            if (left) {
                const int kk = __builtin_ctz(left);
                left &= left - 1u;
                R x = vx[0], y = vy[0], z = vz[0];
#pragma unroll
                for (int k = 1; k < K; ++k)
                    if (kk == k) {
                        x = vx[k];
                        y = vy[k];
                        z = vz[k];
                    }
                mcc_scatter<R>(x, y, z, pid_s[threadIdx.x + kk * T], a.seed, step, a.mass_ratio);
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (kk == k) {
                        vx[k] = x;
                        vy[k] = y;
                        vz[k] = z;
                    }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = threadIdx.x + k * T;
        if (i < (int)n && !((edge >> k) & 1u)) {
            const int32_t g = orig[i];
            vx_g[g] = vx[k];
            vy_g[g] = vy[k];
            vz_g[g] = vz[k];
        }
    }
    // every thread leaves together (see cell_pass)
    __syncthreads();
}

template <typename R, int T, int K, int F>
__global__ __launch_bounds__(T) void k_seg_collide(CollideArgs a, const int32_t *__restrict__ list,
                                                   SegScratch ss)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t wtot[T / PIC_WAVE];
    __shared__ int s_item;
    if (gated_off(a)) return;
    const uint32_t count = a.dflags->count[SEG_SLOT];
    if (blockIdx.x >= count) return;   // no work for this workgroup (nor a queue atomic)
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(&a.dflags->head[SEG_SLOT], 1u);
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item >= (int)count) break;
        seg_pass<R, T, K, F>(a, list, ss, item, smem, wtot);
    }
}

// The pairs across segment edges: the lower member (even position) is the
// last of the previous non-empty segment of the cell, the upper one the first
// of this segment; both are still unchanged.  Rotation, the null collisions of
// both, stores.
template <typename R>
__global__ __launch_bounds__(256) void k_seg_fixup(CollideArgs a, const int32_t *__restrict__ list,
                                                   SegScratch ss)
{
    if (gated_off(a)) return;
    const uint32_t nseg = a.dflags->count[SEG_SLOT];
    const uint32_t step = (uint32_t)read_step(a);
    R *vx_g = (R *)a.v;
    R *vy_g = vx_g + a.n;
    R *vz_g = vy_g + a.n;
    const R *mx = (const R *)ss.m_v;
    const R *my = mx + ss.m_stride;
    const R *mz = my + ss.m_stride;
    for (uint32_t seg = blockIdx.x * blockDim.x + threadIdx.x; seg < nseg; seg += gridDim.x * blockDim.x) {
        const int32_t sb = ss.bnd_head[seg];
        if (sb < 0) continue;
        const int h = ss.sg_cell[seg];
        if (ss.hc_fb[h]) continue;
        int32_t sa = -1;
        for (int p = (int)seg - 1; p >= ss.hc_seg[h]; --p)
            if (ss.sg_cnt[p]) {
                sa = ss.bnd_tail[p];
                break;
            }
        if (sa < 0) continue;   // not reached: an odd offset follows a segment that ends on an even one
        const R C = (R)cell_C(a, list[h]);
        const uint32_t pa = ss.m_pid[sa], pb = ss.m_pid[sb];
        const W4 wa = draw4(a.seed, pa, step, 0u, 0u);
        const W4 wb = draw4(a.seed, pb, step, 0u, 0u);
        R ax = mx[sa], ay = my[sa], az = mz[sa];
        R bx = mx[sb], by = my[sb], bz = mz[sb];
        R hx, hy, hz;
        ta_half(ax - bx, ay - by, az - bz, C, wa.z, wa.w, wb.z, hx, hy, hz);
        ax += hx;
        ay += hy;
        az += hz;
        bx -= hx;
        by -= hy;
        bz -= hz;
        if (a.mcc_thr && (uint64_t)wa.y < a.mcc_thr) mcc_scatter<R>(ax, ay, az, pa, a.seed, step, a.mass_ratio);
        if (a.mcc_thr && (uint64_t)wb.y < a.mcc_thr) mcc_scatter<R>(bx, by, bz, pb, a.seed, step, a.mass_ratio);
        const int32_t ga = ss.m_orig[sa], gb = ss.m_orig[sb];
        vx_g[ga] = ax;
        vy_g[ga] = ay;
        vz_g[ga] = az;
        vx_g[gb] = bx;
        vy_g[gb] = by;
        vz_g[gb] = bz;
    }
}

// ------------------------------------------------------------ deferred cells
// A cell the gate defers skips the Coulomb step and enters no class queue.
// When null collisions are on it is listed here for its candidates (about 1%
// of the members: one Philox word per member decides).  One workgroup per
// cell, cells dealt round-robin (no queue atomics).
constexpr int DEFER_T = 256;

template <typename R>
__global__ __launch_bounds__(DEFER_T) void k_deferred(CollideArgs a, const int32_t *__restrict__ list)
{
    if (gated_off(a)) return;
    const uint32_t count = a.dflags->count[LIST_DEFERRED];
    const uint32_t step = (uint32_t)read_step(a);
    for (uint32_t item = blockIdx.x; item < count; item += gridDim.x) {
        const int cell = list[item];
        const int lo = a.cell_start[cell];
        const int n = a.cell_start[cell + 1] - lo;
        R *vx_g = (R *)a.v + lo;
        R *vy_g = (R *)a.v + a.n + lo;
        R *vz_g = (R *)a.v + 2 * a.n + lo;
        const uint32_t *pid_c = a.pid + lo;
        for (int i = threadIdx.x; i < n; i += DEFER_T) {
            if ((uint64_t)draw4(a.seed, pid_c[i], step, 0u, 0u).y < a.mcc_thr) {
                R x = vx_g[i], y = vy_g[i], z = vz_g[i];
                mcc_scatter<R>(x, y, z, pid_c[i], a.seed, step, a.mass_ratio);
                vx_g[i] = x;
                vy_g[i] = y;
                vz_g[i] = z;
            }
        }
    }
}

// ------------------------------------------------------------ class table
// Class c handles cells with at most cap[c] members (T threads x K items).
template <typename R> struct Classes;
template <> struct Classes<float> {
    static constexpr int T0 = 256, K0 = 2;    // <= 512
    static constexpr int T1 = 512, K1 = 4;    // <= 2048
    // 512 x 8 rather than 1024 x 4: two workgroups (74 KB of LDS each) are
    // resident per CU, and one hides the other's latencies
    static constexpr int T2 = 512, K2 = 8;    // <= 4096
    static constexpr int T3 = 1024, K3 = 10;  // <= 10240
};
template <> struct Classes<double> {
    static constexpr int T0 = 256, K0 = 2;
    static constexpr int T1 = 512, K1 = 4;
    static constexpr int T2 = 1024, K2 = 4;
    static constexpr int T3 = 1024, K3 = 6;   // <= 6144
};
static_assert(Classes<float>::T3 * Classes<float>::K3 == PIC_NOALLOC_MAX_CELL_F32 &&
                  Classes<double>::T3 * Classes<double>::K3 == PIC_NOALLOC_MAX_CELL_F64,
              "the allocation-free step takes the cells of the LDS classes");

// The binary64 lean pass: 1,024 threads of ten members (cells of up to
// 10,240 members on one workgroup instead of the segmented path).
constexpr int LEAN64_T = 1024, LEAN64_K = 10;

// Workgroup geometry of one segment of the segmented path: the largest
// class's (segments of 2,560 members on two 512-thread workgroups per CU
// were slower: more segments, histograms and edge pairs).
template <typename R> struct SegGeom;
template <> struct SegGeom<float> {
    static constexpr int T = 1024, K = 10, PER_CU = 1;
};
template <> struct SegGeom<double> {
    static constexpr int T = 1024, K = 6, PER_CU = 1;
};

// ------------------------------------------------------------ one wave per cell
// Small cells on a single wave with its own slice of LDS: the same pairing,
// rotation and null collisions as the block passes, with wave-level
// synchronisation only (LDS operations of one wave complete in order), so the
// 16 waves of a workgroup work on 16 cells at once.
template <typename R> struct WaveGeom;
template <> struct WaveGeom<float> {
    static constexpr int KW = 8;       // cells of up to 512 members
};
template <> struct WaveGeom<double> {
    static constexpr int KW = 4;       // up to 256 (records of 32 bytes)
};
constexpr size_t WAVE_SLICE = 8 * 1024 + 512;   // LDS bytes per wave

__device__ __forceinline__ void wave_sync()
{
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

template <typename R, bool MCC>
__device__ __forceinline__ void wave_pass(const CollideArgs &a, int cell, unsigned char *slice)
{
    constexpr int KW = WaveGeom<R>::KW;
    constexpr int CAP = PIC_WAVE * KW;
    const int lane = threadIdx.x & (PIC_WAVE - 1);
    const int lo = a.cell_start[cell];
    const int n = a.cell_start[cell + 1] - lo;
    if (n == 0) return;
    const uint32_t step = (uint32_t)read_step(a);
    R *vx_g = (R *)a.v + lo;
    R *vy_g = (R *)a.v + a.n + lo;
    R *vz_g = (R *)a.v + 2 * a.n + lo;
    const uint32_t *pid_c = a.pid + lo;
    R vx[KW], vy[KW], vz[KW];
    uint32_t w2[KW], w3[KW], key[KW], pos[KW];
    uint32_t cand = 0, multi = 0;
    {
        int ic[KW];
#pragma unroll
        for (int k = 0; k < KW; ++k) ic[k] = min(lane + k * PIC_WAVE, n - 1);
#pragma unroll
        for (int k = 0; k < KW; ++k) pos[k] = pid_c[ic[k]];
        asm volatile("" ::: "memory");   // keep the id loads ahead of the velocity loads
#pragma unroll
        for (int k = 0; k < KW; ++k) {
            vx[k] = vx_g[ic[k]];
            vy[k] = vy_g[ic[k]];
            vz[k] = vz_g[ic[k]];
        }
    }
    if (n >= 2) {
        const uint32_t bits = sort_bits(n);
        const uint32_t nb = 1u << bits;
        uint32_t *cnt = (uint32_t *)slice;
        uint32_t *sk = cnt + CAP + 4;
        uint16_t *lst = (uint16_t *)(sk + CAP);
        for (uint32_t q = lane; q < nb; q += PIC_WAVE) cnt[q] = 0u;
        wave_sync();
#pragma unroll
        for (int k = 0; k < KW; ++k) {
            const int i = lane + k * PIC_WAVE;
            if (i < n) {
                const W4 w = draw4(a.seed, pos[k], step, 0u, 0u);
                key[k] = w.x;
                w2[k] = w.z;
                w3[k] = w.w;
                if (MCC && (uint64_t)w.y < a.mcc_thr) cand |= 1u << k;
                pos[k] = atomicAdd(&cnt[w.x >> (32u - bits)], 1u);
            }
        }
        wave_sync();
        {
            // bucket starts: rows of 64 counters with a running carry
            uint32_t carry = 0;
            for (uint32_t r0 = 0; r0 < nb; r0 += PIC_WAVE) {
                const uint32_t q = r0 + lane;
                const uint32_t v = q < nb ? cnt[q] : 0u;
                const uint32_t inc = wave_incl_scan_dpp(v);
                if (q < nb) cnt[q] = carry + inc - v;
                carry += (uint32_t)__builtin_amdgcn_readlane((int)inc, PIC_WAVE - 1);
            }
            if (lane == 0) cnt[nb] = carry;
        }
        wave_sync();
#pragma unroll
        for (int k = 0; k < KW; ++k) {
            const int i = lane + k * PIC_WAVE;
            if (i < n) {
                const uint32_t b = key[k] >> (32u - bits);
                const uint32_t st = cnt[b], en = cnt[b + 1];
                const uint32_t slot = st + pos[k];
                pos[k] = slot;
                if (en - st > 1u) {
                    multi |= 1u << k;
                    sk[slot] = key[k];
                    lst[slot] = (uint16_t)i;
                }
            }
        }
        wave_sync();
#pragma unroll
        for (int k = 0; k < KW; ++k) {
            if ((multi >> k) & 1u) {
                const int i = lane + k * PIC_WAVE;
                const uint32_t b = key[k] >> (32u - bits);
                const uint32_t st = cnt[b], en = cnt[b + 1];
                uint32_t r = 0, tie = 0;
                for (uint32_t j = st; j < en; ++j) {
                    const uint32_t kj = sk[j];
                    r += kj < key[k] ? 1u : 0u;
                    tie |= (kj == key[k] && j != pos[k]) ? 1u : 0u;
                }
                if (tie) {
                    const uint32_t pi = pid_c[i];
                    for (uint32_t j = st; j < en; ++j)
                        if (j != pos[k] && sk[j] == key[k] && pid_c[lst[j]] < pi) ++r;
                }
                pos[k] = st + r;
            }
        }
        wave_sync();   // the sort's slice becomes the exchange records
        const R C = (R)cell_C(a, cell);
        const uint32_t np2 = (uint32_t)n & ~1u;
        Rec<R> *rec = (Rec<R> *)slice;
#pragma unroll
        for (int k = 0; k < KW; ++k) {
            const int i = lane + k * PIC_WAVE;
            if (i < n && pos[k] < np2) {
                Rec<R> e;
                e.x = vx[k];
                e.y = vy[k];
                e.z = vz[k];
                if constexpr (std::is_same<R, float>::value) {
                    // first members carry their deviate, second ones word 2
                    e.w2 = (pos[k] & 1u) ? w2[k] : __float_as_uint(ta_z(w2[k], w3[k]));
                } else {
                    e.w2 = w2[k];
                    e.pad = w3[k];
                }
                rec[pos[k]] = e;
            }
        }
        wave_sync();
        for (uint32_t j = lane; j < np2 / 2; j += PIC_WAVE) {
            Rec<R> A = rec[2 * j], B = rec[2 * j + 1];
            R hx, hy, hz;
            if constexpr (std::is_same<R, float>::value)
                ta_half_z(A.x - B.x, A.y - B.y, A.z - B.z, C, __uint_as_float(A.w2), B.w2, hx, hy, hz);
            else
                ta_half(A.x - B.x, A.y - B.y, A.z - B.z, C, A.w2, A.pad, B.w2, hx, hy, hz);
            A.x += hx;
            A.y += hy;
            A.z += hz;
            B.x -= hx;
            B.y -= hy;
            B.z -= hz;
            rec[2 * j] = A;
            rec[2 * j + 1] = B;
        }
        wave_sync();
#pragma unroll
        for (int k = 0; k < KW; ++k) {
            const int i = lane + k * PIC_WAVE;
            if (i < n && pos[k] < np2) {
                const Rec<R> e = rec[pos[k]];
                vx[k] = e.x;
                vy[k] = e.y;
                vz[k] = e.z;
            }
        }
    } else if (MCC) {
        const W4 w = draw4(a.seed, pos[0], step, 0u, 0u);
        if (lane == 0 && (uint64_t)w.y < a.mcc_thr) cand = 1u;
    }
    if constexpr (MCC) {
        uint32_t left = cand;
        while (__ballot(left != 0u) != 0ull) {
            if (left) {
                const int kk = __builtin_ctz(left);
                left &= left - 1u;
                R x = vx[0], y = vy[0], z = vz[0];
#pragma unroll
                for (int k = 1; k < KW; ++k)
                    if (kk == k) {
                        x = vx[k];
                        y = vy[k];
                        z = vz[k];
                    }
                mcc_scatter<R>(x, y, z, pid_c[lane + kk * PIC_WAVE], a.seed, step, a.mass_ratio);
#pragma unroll
                for (int k = 0; k < KW; ++k)
                    if (kk == k) {
                        vx[k] = x;
                        vy[k] = y;
                        vz[k] = z;
                    }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < KW; ++k) {
        const int i = lane + k * PIC_WAVE;
        if (i < n) {
            vx_g[i] = vx[k];
            vy_g[i] = vy[k];
            vz_g[i] = vz[k];
        }
    }
    wave_sync();   // the slice is free for the wave's next cell
}

// ------------------------------------------------------------ one launch per step
// The block cells of the step (every class that a whole workgroup takes, and
// with the wave schedule off also the smallest class) in one list ordered
// largest first: a counting sort of the cells by a size bucket that halves
// every four steps (sizes within a bucket differ by at most 19%).  One
// workgroup; order[] gets the cells, flags->pad[ORDER_TOTAL] their number.
constexpr int ORDER_BUCKETS = 72;
constexpr int ORDER_TOTAL = 0;   // index into DevFlags::pad

__device__ __forceinline__ int order_bucket(int32_t n)
{
    // 4 log2 n rounded down, from the leading bit and the two bits after it
    const uint32_t u = n > 1 ? (uint32_t)n : 1u;
    const int msb = 31 - __clz(u);
    const int frac = msb >= 2 ? (int)((u >> (msb - 2)) & 3u) : (int)((u << (2 - msb)) & 3u);
    const int key = 4 * msb + frac;                 // grows with n
    const int b = ORDER_BUCKETS - 1 - key;          // largest first
    return b < 0 ? 0 : b;
}

__global__ __launch_bounds__(1024) void k_order_queue(const int32_t *__restrict__ cs,
                                                      const int32_t *__restrict__ lists, int32_t M,
                                                      int first_cls, int last_cls, DevFlags *f,
                                                      int32_t *__restrict__ order)
{
    __shared__ uint32_t hist[ORDER_BUCKETS];
    __shared__ uint32_t cls_off[5];
    if (threadIdx.x < ORDER_BUCKETS) hist[threadIdx.x] = 0u;
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int c = first_cls; c <= last_cls; ++c) {
            cls_off[c] = acc;
            acc += f->count[c];
        }
        cls_off[4] = acc;
        f->pad[ORDER_TOTAL] = acc;
    }
    __syncthreads();
    const uint32_t total = cls_off[4];
    // the cells of classes first..last, walked as one run
    auto cell_at = [&](uint32_t q) {
        int c = first_cls;
        while (c < last_cls && q >= cls_off[c + 1]) ++c;
        return lists[(int64_t)c * M + (q - cls_off[c])];
    };
    for (uint32_t q = threadIdx.x; q < total; q += 1024) {
        const int32_t cell = cell_at(q);
        atomicAdd(&hist[order_bucket(cs[cell + 1] - cs[cell])], 1u);
    }
    __syncthreads();
    if (threadIdx.x < PIC_WAVE) {
        uint32_t carry = 0;
        for (int b0 = 0; b0 < ORDER_BUCKETS; b0 += PIC_WAVE) {
            const int b = b0 + (int)threadIdx.x;
            const uint32_t v = b < ORDER_BUCKETS ? hist[b] : 0u;
            const uint32_t inc = wave_incl_scan(v);
            if (b < ORDER_BUCKETS) hist[b] = carry + inc - v;
            carry += __shfl(inc, PIC_WAVE - 1, PIC_WAVE);
        }
    }
    __syncthreads();
    for (uint32_t q = threadIdx.x; q < total; q += 1024) {
        const int32_t cell = cell_at(q);
        order[atomicAdd(&hist[order_bucket(cs[cell + 1] - cs[cell])], 1u)] = cell;
    }
}

// The whole collide pass of a step in one persistent launch: each workgroup
// takes items from one queue, the segments of the largest cells first, then
// the block cells largest first (their size picks the pass: 1024 threads with
// K members each), and when that queue is empty each of its waves takes cells
// of the smallest class one at a time.  Small cells thus fill the tail that
// the large ones leave, inside the same launch.
template <typename R, int F>
__global__ __launch_bounds__(1024) void k_collide_all(CollideArgs a, const int32_t *__restrict__ lists,
                                                      int32_t M, const int32_t *__restrict__ order,
                                                      SegScratch ss, ClassCaps caps, int use_seg,
                                                      int wave_cls)
{
    constexpr bool MCC = (F & F_MCC) != 0;
    typedef Classes<R> CL;
    typedef SegGeom<R> SG;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t wtot[16];
    __shared__ int s_item;
    if (gated_off(a)) return;
    const uint32_t nseg = use_seg ? a.dflags->count[SEG_SLOT] : 0u;
    const uint32_t nblk = nseg + a.dflags->pad[ORDER_TOTAL];
    const int32_t *l4 = lists + (int64_t)4 * M;
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(&a.dflags->head[0], 1u);
        lds_barrier();   // the previous cell's stores stay in flight
        const uint32_t item = (uint32_t)s_item;
        lds_barrier();
        if (item >= nblk) break;
        if (item < nseg) {
            seg_pass<R, SG::T, SG::K, F>(a, l4, ss, (int)item, smem, wtot);
            continue;
        }
        const int cell = order[item - nseg];
        const int n = a.cell_start[cell + 1] - a.cell_start[cell];
        if constexpr (std::is_same<R, float>::value && (F & ~F_MCC) == 0) {
            // one geometry for every block cell (a second one in the same
            // kernel pushes the largest past the register file)
            (void)n;
            lean_pass<1024, CL::K3, MCC>(a, cell, smem, wtot);
        } else {
            __shared__ double red[16 * 16];
            __shared__ double s_before[4];
            if (n <= 2048) cell_pass<R, 1024, 2, F>(a, cell, smem, red, wtot, s_before);
            else if (n <= 4096) cell_pass<R, 1024, 4, F>(a, cell, smem, red, wtot, s_before);
            else cell_pass<R, 1024, CL::K3, F>(a, cell, smem, red, wtot, s_before);
        }
    }
    if (wave_cls < 0) return;
    // wave phase: one cell per wave, no workgroup barriers from here on
    const uint32_t nw = a.dflags->count[wave_cls];
    const int32_t *wl = lists + (int64_t)wave_cls * M;
    unsigned char *slice = smem + (threadIdx.x / PIC_WAVE) * WAVE_SLICE;
    for (;;) {
        uint32_t item = 0;
        if ((threadIdx.x & (PIC_WAVE - 1)) == 0) item = atomicAdd(&a.dflags->head[1], 1u);
        item = (uint32_t)__builtin_amdgcn_readfirstlane((int)__shfl(item, 0, PIC_WAVE));
        if (item >= nw) break;
        wave_pass<R, MCC>(a, wl[item], slice);
    }
}

template <typename R, int T, int K, int F>
int launch_class(const CollideArgs &a, const int32_t *list, int cls, int blocks, hipStream_t st)
{
    const size_t lds = lds_bytes<R, F>(T * K);
    auto kern = k_collide<R, T, K, F>;
    static bool attr_done = false;
    if (!attr_done) {
        HIP_OK(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds));
        attr_done = true;
    }
    ktime_begin(KT_CLASS0 + cls, st);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(T), lds, st, a, list, cls);
    ktime_end(KT_CLASS0 + cls, st);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

// The lean pass for binary32 steps without conservation sums, moment sums or
// the pairing export; cell_pass otherwise.
template <typename R, int T, int K, int F>
int launch_class_best(const CollideArgs &a, const int32_t *list, int cls, int blocks, hipStream_t st)
{
    if constexpr (std::is_same<R, float>::value && (F & ~F_MCC) == 0) {
        constexpr bool MCC = (F & F_MCC) != 0;
        const size_t lds = lean_lds_bytes<T, K>();
        auto kern = k_collide_lean<T, K, MCC>;
        static bool attr_done = false;
        if (!attr_done) {
            HIP_OK(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds));
            attr_done = true;
        }
        ktime_begin(KT_CLASS0 + cls, st);
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(T), lds, st, a, list, cls);
        ktime_end(KT_CLASS0 + cls, st);
        HIP_OK(hipGetLastError());
        return PIC_OK;
    } else {
        return launch_class<R, T, K, F>(a, list, cls, blocks, st);
    }
}

template <bool MCC, int K = LEAN64_K>
int launch_lean64(const CollideArgs &a, const int32_t *list, int cls, int blocks, hipStream_t st)
{
    constexpr int T = LEAN64_T;
    const size_t lds = lean64_lds_bytes<T, K>();
    auto kern = k_collide_lean64<T, K, MCC>;
    static bool attr_done = false;
    if (!attr_done) {
        HIP_OK(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr_done = true;
    }
    ktime_begin(KT_CLASS0 + cls, st);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(T), lds, st, a, list, cls);
    ktime_end(KT_CLASS0 + cls, st);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

SegScratch g_seg;   // set from the workspace before each step's launches

template <typename R, int T, int K, int F>
int launch_seg_collide(const CollideArgs &a, const int32_t *list, const SegScratch &ss, int blocks,
                       hipStream_t st)
{
    const size_t lds = lds_bytes<R>(T * K);
    auto kern = k_seg_collide<R, T, K, F>;
    static bool attr_done = false;
    if (!attr_done) {
        HIP_OK(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds));
        attr_done = true;
    }
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(T), lds, st, a, list, ss);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

template <typename R, int F>
int launch_all(const CollideArgs &a, const int32_t *lists, int32_t n_cells, int num_cu,
               const HugeScratch &hs, const ClassCaps &caps, bool seg_path, uint32_t live,
               hipStream_t st)
{
    typedef Classes<R> C;
    constexpr bool PAIRS = (F & F_PAIRS) != 0;
    constexpr bool SEG_OK = !PAIRS && !(F & (F_CONS | F_MOM | F_WT | F_NANBU | F_TRIP));
    int rc;
    const int64_t M = n_cells;
    const int *bp = caps.blocks_per_cu;
    const int32_t *l4 = lists + 4 * M;
    // largest cells first so the small ones fill the tail
    ktime_begin(KT_HUGE, st);
    bool seg_done = !(live & (1u << 4));   // no cell beyond the LDS classes
    if constexpr (SEG_OK) {
      if (!seg_done && seg_path) {
        seg_done = true;
        const SegScratch &ss = g_seg;
        hipLaunchKernelGGL(k_seg_count, dim3(num_cu * 4), dim3(SEG_CT), 0, st, a, l4, ss);
        typedef SegGeom<R> G;
        hipLaunchKernelGGL(k_seg_scan, dim3(1), dim3(1024), 0, st, a, ss, (uint32_t)(G::T * G::K));
        hipLaunchKernelGGL(k_seg_scatter<R>, dim3(num_cu * 4), dim3(SEG_CT), 0, st, a, l4, ss);
        HIP_OK(hipGetLastError());
        if ((rc = launch_seg_collide<R, G::T, G::K, F>(a, l4, ss, G::PER_CU * num_cu, st))) return rc;
        hipLaunchKernelGGL(k_seg_fixup<R>, dim3(num_cu), dim3(256), 0, st, a, l4, ss);
        // cells the plan could not segment
        hipLaunchKernelGGL((k_collide_huge<R, PAIRS>), dim3(num_cu * bp[4]), dim3(1024), 0, st, a, l4, 4,
                           hs, (const uint8_t *)ss.hc_fb);
      }
    }
    if (!seg_done)
        hipLaunchKernelGGL((k_collide_huge<R, PAIRS>), dim3(num_cu * bp[4]), dim3(1024), 0, st, a, l4, 4,
                           hs, (const uint8_t *)nullptr);
    ktime_end(KT_HUGE, st);
    HIP_OK(hipGetLastError());
    if (live & (1u << 3)) {
        // binary64 plain steps whose caps widen the largest class: the lean pass
        bool done = false;
        if constexpr (std::is_same<R, double>::value && (F & ~F_MCC) == 0) {
            if (caps.cap[3] > C::T3 * C::K3) {
                // one workgroup per listed cell (the kernel is not persistent)
                if ((rc = launch_lean64<(F & F_MCC) != 0>(a, lists + 3 * M, 3, (int)M, st)))
                    return rc;
                done = true;
            }
        }
        if (!done &&
            (rc = launch_class_best<R, C::T3, C::K3, F>(a, lists + 3 * M, 3, bp[3] * num_cu, st)))
            return rc;
    }
    if (live & (1u << 2)) {
        bool done = false;
        if constexpr (std::is_same<R, double>::value && (F & ~F_MCC) == 0) {
            if (caps.cap[3] > C::T3 * C::K3) {   // the binary64 plain step's lean passes
                if ((rc = launch_lean64<(F & F_MCC) != 0, C::K2>(a, lists + 2 * M, 2, (int)M, st)))
                    return rc;
                done = true;
            }
        }
        if (!done &&
            (rc = launch_class_best<R, C::T2, C::K2, F>(a, lists + 2 * M, 2, bp[2] * num_cu, st)))
            return rc;
    }
    if ((live & (1u << 1)) &&
        (rc = launch_class_best<R, C::T1, C::K1, F>(a, lists + 1 * M, 1, bp[1] * num_cu, st)))
        return rc;
    if ((live & (1u << 0)) &&
        (rc = launch_class<R, C::T0, C::K0, F>(a, lists + 0 * M, 0, bp[0] * num_cu, st)))
        return rc;
    return PIC_OK;
}

// Dynamic LDS of the one-launch pass: the largest of its block passes and the
// waves' slices.
template <typename R, int F>
constexpr size_t all_lds_bytes()
{
    typedef Classes<R> CL;
    size_t b = 16 * WAVE_SLICE;
    const size_t seg = lds_bytes<R>(SegGeom<R>::T * SegGeom<R>::K);
    b = seg > b ? seg : b;
    if constexpr (std::is_same<R, float>::value && (F & ~F_MCC) == 0) {
        const size_t l = lean_lds_bytes<1024, CL::K3>();
        b = l > b ? l : b;
    } else {
        const size_t l = lds_bytes<R>(1024 * CL::K3);
        b = l > b ? l : b;
    }
    return b;
}

// The step's collide pass as one persistent launch (see k_collide_all): the
// segment pre-passes of the cells beyond the LDS classes, the largest-first
// order of the block cells, the launch, then the pairs across segment edges
// and the cells no segment plan could take.
template <typename R, int F>
int launch_unified(const CollideArgs &a, const int32_t *lists, int32_t n_cells, int num_cu,
                   const HugeScratch &hs, const ClassCaps &caps, bool seg_path, hipStream_t st)
{
    const int32_t *l4 = lists + 4 * (int64_t)n_cells;
    const SegScratch &ss = g_seg;
    if (seg_path) {
        ktime_begin(KT_HUGE, st);
        hipLaunchKernelGGL(k_seg_count, dim3(num_cu * 4), dim3(SEG_CT), 0, st, a, l4, ss);
        typedef SegGeom<R> G;
        hipLaunchKernelGGL(k_seg_scan, dim3(1), dim3(1024), 0, st, a, ss, (uint32_t)(G::T * G::K));
        hipLaunchKernelGGL(k_seg_scatter<R>, dim3(num_cu * 4), dim3(SEG_CT), 0, st, a, l4, ss);
        ktime_end(KT_HUGE, st);
    }
    const int wave_cls = caps.wave ? 0 : -1;
    ktime_begin(KT_QUEUE, st);
    hipLaunchKernelGGL(k_order_queue, dim3(1), dim3(1024), 0, st, a.cell_start, lists, n_cells,
                       caps.wave ? 1 : 0, caps.ncls - 1, a.dflags, a.order);
    ktime_end(KT_QUEUE, st);
    constexpr size_t lds = all_lds_bytes<R, F>();
    auto kern = k_collide_all<R, F>;
    static bool attr_done = false;
    if (!attr_done) {
        HIP_OK(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds));
        attr_done = true;
    }
    ktime_begin(KT_ALL, st);
    hipLaunchKernelGGL(kern, dim3(num_cu), dim3(1024), lds, st, a, lists, n_cells,
                       (const int32_t *)a.order, ss, caps, seg_path ? 1 : 0, wave_cls);
    ktime_end(KT_ALL, st);
    HIP_OK(hipGetLastError());
    ktime_begin(KT_HUGE, st);
    if (seg_path) {
        hipLaunchKernelGGL(k_seg_fixup<R>, dim3(num_cu), dim3(256), 0, st, a, l4, ss);
        hipLaunchKernelGGL((k_collide_huge<R, false>), dim3(num_cu), dim3(1024), 0, st, a, l4, 4, hs,
                           (const uint8_t *)ss.hc_fb);
    } else {
        hipLaunchKernelGGL((k_collide_huge<R, false>), dim3(num_cu), dim3(1024), 0, st, a, l4, 4, hs,
                           (const uint8_t *)nullptr);
    }
    ktime_end(KT_HUGE, st);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

template <typename R>
int launch_deferred_t(const CollideArgs &a, const int32_t *lists, int32_t n_cells, int num_cu,
                      hipStream_t st)
{
    const int g = n_cells < num_cu * 8 ? n_cells : num_cu * 8;
    hipLaunchKernelGGL(k_deferred<R>, dim3(g), dim3(DEFER_T), 0, st, a,
                       lists + (int64_t)LIST_DEFERRED * n_cells);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

template <typename R>
int launch_flags(const CollideArgs &a, const int32_t *lists, int32_t n_cells, int num_cu,
                 const HugeScratch &hs, const ClassCaps &cc, int pairs_only, bool sp, uint32_t lv,
                 hipStream_t st)
{
    if (pairs_only) return launch_all<R, F_PAIRS>(a, lists, n_cells, num_cu, hs, cc, false, ~0u, st);
    if (a.variant == VAR_NANBU) return launch_all<R, F_NANBU>(a, lists, n_cells, num_cu, hs, cc, false, lv, st);
    if (a.variant == VAR_TRIPLET) return launch_all<R, F_TRIP>(a, lists, n_cells, num_cu, hs, cc, false, lv, st);
    if (a.w) {
        // variable weights: the plain step (optionally with null collisions),
        // cells beyond the LDS classes on one workgroup each
        if (a.mcc_thr) return launch_all<R, F_WT | F_MCC>(a, lists, n_cells, num_cu, hs, cc, false, lv, st);
        return launch_all<R, F_WT>(a, lists, n_cells, num_cu, hs, cc, false, lv, st);
    }
    const int f = (a.mcc_thr ? F_MCC : 0) | ((a.flags & PIC_CONSERVE_FIX) ? F_CONS : 0) |
                  ((a.flags & PIC_MOMENTS) ? F_MOM : 0);
    // the plain step (with or without null collisions) as one launch
    if (cc.unified && a.order && (f & ~F_MCC) == 0)
        return f ? launch_unified<R, F_MCC>(a, lists, n_cells, num_cu, hs, cc, sp, st)
                 : launch_unified<R, 0>(a, lists, n_cells, num_cu, hs, cc, sp, st);
    switch (f) {
    case 0: return launch_all<R, 0>(a, lists, n_cells, num_cu, hs, cc, sp, lv, st);
    case 1: return launch_all<R, 1>(a, lists, n_cells, num_cu, hs, cc, sp, lv, st);
    case 2: return launch_all<R, 2>(a, lists, n_cells, num_cu, hs, cc, sp, lv, st);
    case 3: return launch_all<R, 3>(a, lists, n_cells, num_cu, hs, cc, sp, lv, st);
    case 4: return launch_all<R, 4>(a, lists, n_cells, num_cu, hs, cc, sp, lv, st);
    case 5: return launch_all<R, 5>(a, lists, n_cells, num_cu, hs, cc, sp, lv, st);
    case 6: return launch_all<R, 6>(a, lists, n_cells, num_cu, hs, cc, sp, lv, st);
    default: return launch_all<R, 7>(a, lists, n_cells, num_cu, hs, cc, sp, lv, st);
    }
}

HugeScratch g_huge;   // set by launch_collide from the workspace

}  // namespace

const HugeScratch &huge_scratch() { return g_huge; }

namespace {


}  // namespace

ClassCaps collide_caps(int dtype, size_t)
{
    ClassCaps c;
    c.ncls = 4;
    // one launch per size class by default: measured faster than the single
    // persistent launch on the uniform and the log-normal workloads (the
    // autotuner tries both)
    c.unified = 0;
    c.wave = 1;
    c.blocks_per_cu[0] = 8;
    c.blocks_per_cu[1] = 4;
    c.blocks_per_cu[2] = 2;
    c.blocks_per_cu[3] = 1;
    c.blocks_per_cu[4] = 1;
    if (dtype == PIC_F32) {
        typedef Classes<float> C;
        c.cap[0] = C::T0 * C::K0;
        c.cap[1] = C::T1 * C::K1;
        c.cap[2] = C::T2 * C::K2;
        c.cap[3] = C::T3 * C::K3;
    } else {
        typedef Classes<double> C;
        // the wave schedule takes cells of up to 256 members in binary64
        c.cap[0] = PIC_WAVE * WaveGeom<double>::KW;
        c.cap[1] = C::T1 * C::K1;
        c.cap[2] = C::T2 * C::K2;
        c.cap[3] = C::T3 * C::K3;
    }
    return c;
}



int lean64_cap()
{
    return LEAN64_T * LEAN64_K;
}

size_t huge_scratch_bytes(int dtype, int64_t n)
{
    const size_t rec = dtype == PIC_F32 ? 16 : 32;
    return (size_t)n * (4 * 4 + 8 + 1) + ((size_t)n / 2 + 2) * rec + 7 * 256;   // 7 aligned parts
}

void set_huge_scratch(int dtype, int64_t n, void *base)
{
    unsigned char *p = (unsigned char *)base;
    auto take = [&](size_t bytes) {
        unsigned char *r = p;
        p += (bytes + 255) & ~(size_t)255;
        return (void *)r;
    };
    g_huge.keys = (uint32_t *)take((size_t)n * 4);
    g_huge.cnt = (uint32_t *)take((size_t)n * 4);
    g_huge.lst = (uint32_t *)take((size_t)n * 4);
    g_huge.pos = (uint32_t *)take((size_t)n * 4);
    g_huge.w23 = (uint32_t *)take((size_t)n * 8);
    g_huge.cand = (uint8_t *)take((size_t)n);
    g_huge.pbuf = take(((size_t)n / 2 + 2) * (dtype == PIC_F32 ? 16 : 32));
}

int launch_collide(int dtype, const CollideArgs &a, const int32_t *lists, int32_t n_cells,
                   const ClassCaps &cc, int pairs_only, int num_cu, hipStream_t st, bool seg_path,
                   uint32_t live)
{
    if (dtype == PIC_F32)
        return launch_flags<float>(a, lists, n_cells, num_cu, g_huge, cc, pairs_only, seg_path, live, st);
    return launch_flags<double>(a, lists, n_cells, num_cu, g_huge, cc, pairs_only, seg_path, live, st);
}

const SegScratch &seg_scratch() { return g_seg; }

int seg_cap(int dtype)
{
    return dtype == PIC_F32 ? SegGeom<float>::T * SegGeom<float>::K
                            : SegGeom<double>::T * SegGeom<double>::K;
}

int seg_target(int dtype)
{
    return seg_cap(dtype) * 7 / 8;
}

static int64_t seg_max_for(int dtype, int64_t n, int32_t n_cells)
{
    // S = ceil(n_c / target) <= n_c / target + 1 per cell
    return n / seg_target(dtype) + n_cells + 2;
}

static int64_t chunk_max_for(int64_t n, int32_t n_cells)
{
    return n / SEG_CHUNK + n_cells + 1;
}

size_t seg_scratch_bytes(int dtype, int64_t n, int32_t n_cells)
{
    const size_t S = (size_t)seg_max_for(dtype, n, n_cells), Q = (size_t)chunk_max_for(n, n_cells);
    return (size_t)n_cells * (4 + 1 + 4 + 4) + S * 6 * 4 + Q * 4 + 11 * 256;   // 11 aligned parts
}

void set_seg_scratch(int dtype, int64_t n, int32_t n_cells, void *base, int32_t *m_orig,
                     uint32_t *m_pid, void *m_v)
{
    unsigned char *p = (unsigned char *)base;
    auto take = [&](size_t bytes) {
        unsigned char *r = p;
        p += (bytes + 255) & ~(size_t)255;
        return (void *)r;
    };
    const int64_t S = seg_max_for(dtype, n, n_cells), Q = chunk_max_for(n, n_cells);
    g_seg.hc_S = (uint32_t *)take((size_t)n_cells * 4);
    g_seg.hc_fb = (uint8_t *)take((size_t)n_cells);
    g_seg.hc_seg = (int32_t *)take((size_t)n_cells * 4);
    g_seg.hc_chunk = (int32_t *)take((size_t)n_cells * 4);
    g_seg.sg_cell = (int32_t *)take((size_t)S * 4);
    g_seg.sg_cnt = (uint32_t *)take((size_t)S * 4);
    g_seg.sg_start = (uint32_t *)take((size_t)S * 4);
    g_seg.sg_cur = (uint32_t *)take((size_t)S * 4);
    g_seg.bnd_head = (int32_t *)take((size_t)S * 4);
    g_seg.bnd_tail = (int32_t *)take((size_t)S * 4);
    g_seg.ch_owner = (int32_t *)take((size_t)Q * 4);
    g_seg.m_orig = m_orig;
    g_seg.m_pid = m_pid;
    g_seg.m_v = m_v;
    g_seg.m_stride = n;
    g_seg.seg_max = S;
    g_seg.chunk_max = Q;
}

int launch_deferred(int dtype, const CollideArgs &a, const int32_t *lists, int32_t n_cells,
                    int num_cu, hipStream_t st)
{
    if (dtype == PIC_F32) return launch_deferred_t<float>(a, lists, n_cells, num_cu, st);
    return launch_deferred_t<double>(a, lists, n_cells, num_cu, st);
}

// pic_internal.hpp -- device helpers and launch interfaces shared by the
// library's HIP translation units (CDNA4 / gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "piccoll.h"

#define PIC_WAVE 64

// ---------------------------------------------------------------------------
// Device-side status words.  `unsorted` and `range_err` describe the current
// call; the sticky words survive until pic_sync reads and clears them.
// ---------------------------------------------------------------------------
struct DevFlags {
    int unsorted;        // storage not in cell order (re-binning needed)
    int range_err;       // a cell id outside [0, n_cells) in this call
    int sticky_range;    // latched PIC_ERR_RANGE
    int sticky_state;    // latched PIC_ERR_STATE
    int sticky_nonfinite;  // latched PIC_ERR_NONFINITE
    unsigned int head[8];   // work-queue heads of the persistent kernels
    unsigned int count[8];  // work-queue lengths (cells per class)
    unsigned int huge_total; // members of cells in the multi-block class
    unsigned int seg_fallback; // some cell of that class takes the one-workgroup path
    unsigned int pad[5];
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Each round multiplies
// two counter words by the round constants (one 32x32->64 product each),
// mixes the high halves with the other two words and the round key, and the
// key advances by the Weyl increments between rounds.  The key comes from the
// seed and is the same for every lane, so its schedule stays in SGPRs.
// ---------------------------------------------------------------------------
struct W4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ W4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        // three-input exclusive or in one CDNA4 instruction (truth table 0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return W4{c0, c1, c2, c3};
}

__device__ __forceinline__ W4 draw4(uint64_t seed, uint32_t c0, uint32_t step, uint32_t domain,
                                    uint32_t c3)
{
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    // The seed is uniform: keep its round keys in two SGPRs per call.  The
    // empty asm hides the value from the optimiser so the ten round keys of
    // unrolled call sites are not all hoisted and kept live at once.
    asm volatile("" : "+s"(k0), "+s"(k1));
    return philox10(c0, step, domain, c3, k0, k1);
}

// U(x) = ((x >> 9) + 1/2) 2^-23: 24 significant bits, exact in binary32.
__device__ __forceinline__ float u01f(uint32_t x)
{
    return ((float)(x >> 9) + 0.5f) * 0x1p-23f;
}
__device__ __forceinline__ double u01d(uint32_t x)
{
    return ((double)(x >> 9) + 0.5) * 0x1p-23;
}

// Nanbu's Coulomb operator on the pairs of the Takizuka-Abe step: the pair
// (a, b), a the lower slot, turns its relative velocity u by chi with
// 1 - cos chi = -log1p(-(1 - U)(1 - exp(-2A))) / A, U = U(word 2 of a),
// A solving coth A - 1/A = exp(-s), s = 2 * 8 pi n lnL dt / |u|^3; azimuth
// 2 pi U(word 2 of b); halves as in T&A.  Binary64 storage computes in
// binary64 (the oracle's steps exactly); binary32 storage in binary32, with
// the Langevin series used up to A = 0.5 (five terms) where the closed form
// would cancel, and the large-A root up to s = 0.1.
// a / b, correctly rounded in both precisions (the hardware reciprocal's
// extra rounding was enough to miss the binary32 bar where a collision
// leaves a member almost at rest)
template <typename T>
__device__ __forceinline__ T nb_div(T a, T b)
{
    return a / b;
}

template <typename T>
__device__ __forceinline__ void nb_langevin(T A, T &L, T &dL)
{
#pragma clang fp contract(off)
    constexpr bool F = sizeof(T) == 4;
    if (A < (F ? (T)0.5 : (T)0.1)) {
        const T A2 = A * A;
        if (F) {
            L = A * ((T)(1.0 / 3.0) -
                     A2 * ((T)(1.0 / 45.0) - A2 * ((T)(2.0 / 945.0) - A2 * ((T)(1.0 / 4725.0) -
                                                                            A2 * (T)(2.0 / 93555.0)))));
            dL = (T)(1.0 / 3.0) -
                 A2 * ((T)(1.0 / 15.0) - A2 * ((T)(2.0 / 189.0) - A2 * ((T)(1.0 / 675.0) - A2 * (T)(2.0 / 10395.0))));
        } else {
            L = A * (1.0 / 3.0 - A2 * (1.0 / 45.0 - A2 * (2.0 / 945.0 - A2 / 4725.0)));
            dL = 1.0 / 3.0 - A2 * (1.0 / 15.0 - A2 * (2.0 / 189.0 - A2 / 675.0));
        }
    } else {   // t = exp(-2A): coth A = (1 + t)/(1 - t), 1/sinh^2 A = 4t/(1 - t)^2
        const T t = exp((T)-2 * A), d = (T)1 - t;
        L = nb_div((T)1 + t, d) - nb_div((T)1, A);
        dL = nb_div((T)1, A * A) - nb_div((T)4 * t, d * d);
    }
}

template <typename T>
__device__ __forceinline__ T nb_A(T s)
{
#pragma clang fp contract(off)
    // coth A = 1 to working precision: A > 8.3 in binary32, A > 18.7 in binary64
    if (s <= (sizeof(T) == 4 ? (T)0.1 : (T)0.01)) return nb_div((T)-1, expm1(-s));
    const T y = exp(-s);
    if (s > (T)11.5) return (T)3 * y;             // coth A - 1/A = A/3 to 1e-10
    T A = nb_div(y * ((T)3 - y * y), (T)1 - y * y);
    for (int it = 0; it < 4; ++it) {   // from within 2%: quadratic convergence
        T L, dL;
        nb_langevin(A, L, dL);
        A -= nb_div(L - y, dL);
    }
    return A;
}

template <typename T>
__device__ __forceinline__ T nb_omc(T A, T U)
{
#pragma clang fp contract(off)
    if (!(A > (sizeof(T) == 4 ? (T)1e-30 : (T)1e-300))) return (T)2 * ((T)1 - U);
    // -log(U + (1 - U) exp(-2A)) / A: through log1p(-q) while q < 1/2, else
    // the sum itself (no cancellation when U and exp(-2A) are both small)
    const T q = ((T)1 - U) * -expm1((T)-2 * A);
    const T omc = nb_div(q < (T)0.5 ? -log1p(-q) : -log(U + ((T)1 - U) * exp((T)-2 * A)), A);
    return omc < (T)2 ? omc : (T)2;
}


// ---------------------------------------------------------------------------
// Elastic isotropic scattering of a null-collision candidate from its domain-1
// draw w: cos(theta) = 1 - 2 U(w.y), phi = 2 pi U(w.z) (binary32: the hardware
// sine/cosine take revolutions, the hardware square root is within 1 ulp),
// |v'|^2 = |v|^2 (1 - 2 (m/M) (1 - vhat.s)).
// The cross section sigma0 E^-1/2 gives the speed-independent frequency
// nu = n_n sigma0 sqrt(2) = nu_max, so the real/null test U(w.x) nu_max < nu
// always passes and is not evaluated.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void scatter_dir(float &vx, float &vy, float &vz, const W4 &w,
                                            double mass_ratio)
{
    // no contraction: the fused and the stand-alone step round identically
#pragma clang fp contract(off)
    const float ct = 1.0f - 2.0f * u01f(w.y);
    const float st = __builtin_amdgcn_sqrtf(fmaxf(0.0f, 1.0f - ct * ct));
    const float up = u01f(w.z);
    const float sx = st * __builtin_amdgcn_cosf(up), sy = st * __builtin_amdgcn_sinf(up), sz = ct;
    const float sp = __builtin_amdgcn_sqrtf(vx * vx + vy * vy + vz * vz);
    float scale = sp;
    if (mass_ratio != 0.0 && sp > 0.0f) {
        const float cosx = (vx * sx + vy * sy + vz * sz) / sp;
        scale = sp * __builtin_amdgcn_sqrtf(1.0f - 2.0f * (float)mass_ratio * (1.0f - cosx));
    }
    vx = scale * sx;
    vy = scale * sy;
    vz = scale * sz;
}

__device__ __forceinline__ void scatter_dir(double &vx, double &vy, double &vz, const W4 &w,
                                            double mass_ratio)
{
#pragma clang fp contract(off)
    const double ct = 1.0 - 2.0 * u01d(w.y);
    const double st = sqrt(fmax(0.0, 1.0 - ct * ct));
    const double ph = 2.0 * 3.14159265358979323846 * u01d(w.z);
    const double sx = st * cos(ph), sy = st * sin(ph), sz = ct;
    const double sp = sqrt(vx * vx + vy * vy + vz * vz);
    double scale = sp;
    if (mass_ratio != 0.0 && sp > 0.0) {
        const double cosx = (vx * sx + vy * sy + vz * sz) / sp;
        scale = sp * sqrt(1.0 - 2.0 * mass_ratio * (1.0 - cosx));
    }
    vx = scale * sx;
    vy = scale * sy;
    vz = scale * sz;
}

// ---------------------------------------------------------------------------
// Compensated conservation correction of one cell of N members.
// b = (sum v, sum |v|^2) before the Coulomb step, f = the same sums now.  The
// targets are b plus the cell's debt (momentum, sum |v|^2) that earlier steps'
// output rounding left unmet: a binary32 step changes a cell's energy by far
// less than one binary32 ulp, so a plain rescaling would round away and the
// error would accumulate; carrying the shortfall makes it diffuse instead.
// v <- Vt + alpha (v - Vn) with Vt the target mean velocity and alpha^2 the
// ratio of target to current thermal energy.
// ---------------------------------------------------------------------------
struct Correction {
    double Vt[3], Vn[3], al;
    double P[3], Q;   // targets: momentum and sum |v|^2
    bool ok;
};

__device__ __forceinline__ Correction make_correction(double N, const double *b, const double *f,
                                                      const double *debt)
{
    Correction c;
    c.P[0] = b[0];
    c.P[1] = b[1];
    c.P[2] = b[2];
    c.Q = b[3];
    if (debt) {
        c.P[0] += debt[0];
        c.P[1] += debt[1];
        c.P[2] += debt[2];
        c.Q += debt[3];
    }
    double vt2 = 0.0, vn2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        c.Vt[a] = c.P[a] / N;
        c.Vn[a] = f[a] / N;
        vt2 += c.Vt[a] * c.Vt[a];
        vn2 += c.Vn[a] * c.Vn[a];
    }
    const double Et = 0.5 * c.Q - 0.5 * N * vt2;
    const double En = 0.5 * f[3] - 0.5 * N * vn2;
    c.ok = N >= 2.0 && En > 0.0 && Et >= 0.0;
    c.al = c.ok ? sqrt(Et / En) : 1.0;
    return c;
}

// The shortfall left after the correction: target minus the realised sums
// (real[0..2] momentum, real[3] sum |v|^2).
__device__ __forceinline__ void store_debt(double *debt, const Correction &c, const double *real)
{
    debt[0] = c.P[0] - real[0];
    debt[1] = c.P[1] - real[1];
    debt[2] = c.P[2] - real[2];
    debt[3] = c.Q - real[3];
}

// The same from block_sum_scatter<4> totals: thread t < 4 holds realised sum
// t and writes shortfall t.
__device__ __forceinline__ void store_debt_lane(double *debt, const Correction &c, double real_t)
{
    const unsigned t = threadIdx.x;
    if (t < 4) debt[t] = (t == 0 ? c.P[0] : t == 1 ? c.P[1] : t == 2 ? c.P[2] : c.Q) - real_t;
}

// ---------------------------------------------------------------------------
// Wave / block reductions in a fixed order (bitwise reproducible).
// ---------------------------------------------------------------------------
template <typename V>
__device__ __forceinline__ V wave_sum(V x)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, PIC_WAVE);
    return x;
}

// Sum NV doubles over the block; every thread receives the totals.
// red: LDS scratch of NV * (blockDim / 64) doubles.  Contains the barriers.
template <int NV>
__device__ __forceinline__ void block_sum(double (&x)[NV], double *red)
{
    const int lane = threadIdx.x & (PIC_WAVE - 1), wid = threadIdx.x / PIC_WAVE;
    const int nw = blockDim.x / PIC_WAVE;
#pragma unroll
    for (int j = 0; j < NV; ++j) x[j] = wave_sum(x[j]);
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) red[wid * NV + j] = x[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[w * NV + j];
        x[j] = s;
    }
    __syncthreads();
}

// Reduce-scatter butterfly over a wave for NV doubles (NV a power of two
// <= 64): each exchange step halves the values a lane holds (its partner
// keeps the other half), so a wave exchanges NV - 1 + 6 - log2(NV) values
// instead of 6 NV, in a dependent chain of 6 steps.  Lane L ends with the
// wave total of value L >> (6 - log2 NV).  The order of additions is fixed.
// The first two steps (partners 32 and 16 lanes apart) use the CDNA4 lane
// swaps: v_permlane32_swap exchanges the upper half-wave of one register
// with the lower half-wave of another, v_permlane16_swap the odd 16-lane rows
// of one with the even rows of the other; after the swap of (lo, hi) a lane
// in the lower half (rows 0, 2) holds both its own and its partner's lo, one
// in the upper half both hi, and one add finishes the step -- no selects and
// no LDS traffic.  The later steps shuffle.
template <int NV>
constexpr int log2_pow2()
{
    return NV == 1 ? 0 : NV == 2 ? 1 : NV == 4 ? 2 : NV == 8 ? 3 : NV == 16 ? 4 : NV == 32 ? 5 : 6;
}

template <int O>
__device__ __forceinline__ void lane_swap(double &lo, double &hi)
{
    static_assert(O == 32 || O == 16, "lane swaps exist for 32 and 16");
    const uint64_t a = __double_as_longlong(lo), b = __double_as_longlong(hi);
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32), b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
    uint32_t l0, l1, h0, h1;
    if constexpr (O == 32) {
        const auto r0 = __builtin_amdgcn_permlane32_swap(a0, b0, false, false);
        const auto r1 = __builtin_amdgcn_permlane32_swap(a1, b1, false, false);
        l0 = r0[0]; h0 = r0[1]; l1 = r1[0]; h1 = r1[1];
    } else {
        const auto r0 = __builtin_amdgcn_permlane16_swap(a0, b0, false, false);
        const auto r1 = __builtin_amdgcn_permlane16_swap(a1, b1, false, false);
        l0 = r0[0]; h0 = r0[1]; l1 = r1[0]; h1 = r1[1];
    }
    lo = __longlong_as_double((int64_t)(((uint64_t)l1 << 32) | l0));
    hi = __longlong_as_double((int64_t)(((uint64_t)h1 << 32) | h0));
}

// All 64 lanes must be active.
template <int NV>
__device__ __forceinline__ double wave_scatter(double (&x)[NV])
{
    static_assert(NV >= 1 && NV <= PIC_WAVE && (NV & (NV - 1)) == 0, "NV: power of two <= 64");
    constexpr int B = log2_pow2<NV>();
    const int lane = threadIdx.x & (PIC_WAVE - 1);
#pragma unroll
    for (int s = 0; s < B; ++s) {
        const int o = (PIC_WAVE / 2) >> s;
        const int half = NV >> (s + 1);
#pragma unroll
        for (int j = 0; j < half; ++j) {
            if (o == 32 || o == 16) {
                // lower-half lanes: own lo + partner's lo; upper: both hi
                double l = x[j], h = x[j + half];
                if (o == 32) lane_swap<32>(l, h);
                else lane_swap<16>(l, h);
                x[j] = l + h;
            } else {
                const bool up = (lane & o) != 0;
                const double give = up ? x[j] : x[j + half];
                const double keep = up ? x[j + half] : x[j];
                x[j] = keep + __shfl_xor(give, o, PIC_WAVE);
            }
        }
    }
    double v = x[0];
#pragma unroll
    for (int o = (PIC_WAVE >> 1) >> B; o >= 1; o >>= 1) v += __shfl_xor(v, o, PIC_WAVE);
    return v;
}

template <int NV>
__device__ __forceinline__ void wave_scatter_to(double (&x)[NV], double *red)
{
    constexpr int B = log2_pow2<NV>();
    const int lane = threadIdx.x & (PIC_WAVE - 1), wid = threadIdx.x / PIC_WAVE;
    const double v = wave_scatter<NV>(x);
    if ((lane & ((PIC_WAVE >> B) - 1)) == 0) red[wid * NV + (lane >> (6 - B))] = v;
}

// Block totals of NV doubles: thread t < NV returns the total of value t
// (waves added in order), other threads 0.  red: NV * (blockDim / 64)
// doubles of LDS.  Contains the barriers (red is free again on return).
template <int NV>
__device__ __forceinline__ double block_sum_scatter(double (&x)[NV], double *red)
{
    wave_scatter_to<NV>(x, red);
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x < NV) {
        const int nw = blockDim.x / PIC_WAVE;
        for (int w = 0; w < nw; ++w) s += red[w * NV + threadIdx.x];
    }
    __syncthreads();
    return s;
}

// Block totals of NV doubles, returned to every thread in x.  red:
// NV * (blockDim / 64 + 1) doubles of LDS.  Contains the barriers.
template <int NV>
__device__ __forceinline__ void block_sum_bcast(double (&x)[NV], double *red)
{
    const int nw = blockDim.x / PIC_WAVE;
    wave_scatter_to<NV>(x, red);
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[w * NV + threadIdx.x];
        red[nw * NV + threadIdx.x] = s;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; ++j) x[j] = red[nw * NV + j];
    __syncthreads();
}

// Inclusive scan of one uint32 per lane within a wave.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x)
{
    const int lane = threadIdx.x & (PIC_WAVE - 1);
#pragma unroll
    for (int o = 1; o < PIC_WAVE; o <<= 1) {
        uint32_t y = __shfl_up(x, o, PIC_WAVE);
        if (lane >= o) x += y;
    }
    return x;
}

// Block-wide exclusive scan of one value per thread (blockDim <= 1024);
// wtot: LDS scratch of blockDim / 64 words.  Contains two barriers.
__device__ __forceinline__ uint32_t block_excl(uint32_t x, uint32_t *wtot)
{
    const int lane = threadIdx.x & (PIC_WAVE - 1), wid = threadIdx.x / PIC_WAVE;
    const int nw = blockDim.x / PIC_WAVE;
    const uint32_t inc = wave_incl_scan(x);
    if (lane == PIC_WAVE - 1) wtot[wid] = inc;
    __syncthreads();
    uint32_t off = 0;
    for (int w = 0; w < nw; ++w)
        if (w < wid) off += wtot[w];
    __syncthreads();
    return off + inc - x;
}

__device__ __forceinline__ uint32_t get16(const uint32_t *w, uint32_t b)
{
    return (w[b >> 1] >> ((b & 1u) * 16u)) & 0xFFFFu;
}

// ---------------------------------------------------------------------------
// LDS sort of one cell's members by (key, pid).  Buckets are the top `bits`
// bits of the key with nbk = 2^bits >= n buckets (so at most one member per
// bucket on average); the bucket is monotone in the key, so bucket order and
// then (key, pid) order inside a bucket give the full order.  Layout for a
// cell capacity CAP: keys by member, keys in bucket order (padded for 4-wide
// reads), 16-bit bucket counters (two per word), members in bucket order.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr uint32_t next_pow2(uint32_t x)
{
    uint32_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

__host__ __device__ constexpr size_t sort_bytes(int cap)
{
    return (size_t)cap * 4 + ((size_t)cap + 4) * 4 + (size_t)next_pow2((uint32_t)cap) * 2 +
           (size_t)cap * 2;
}

template <int T, int CAP>
struct SortLDS {
    static constexpr int WMAX = (int)(next_pow2(CAP) / 2);   // counter words
    static constexpr int PERW = WMAX / T;                     // words per thread
    static_assert(PERW >= 1 && PERW * T == WMAX, "counter table must split evenly");
    uint32_t *keys;    // [CAP] key of member i
    uint32_t *sk;      // [CAP + 4] keys in bucket order
    uint32_t *cnt;     // [WMAX] bucket counters, then bucket starts
    uint16_t *lst;     // [CAP] member in bucket order
    __device__ explicit SortLDS(unsigned char *smem)
        : keys((uint32_t *)smem), sk(keys + CAP), cnt(sk + CAP + 4), lst((uint16_t *)(cnt + WMAX))
    {
    }
    __device__ uint32_t *own() const { return cnt + threadIdx.x * PERW; }
    // zero the counters (the caller synchronises before counting)
    __device__ void clear() const
    {
        uint32_t *c = own();
#pragma unroll
        for (int q = 0; q < PERW; ++q) c[q] = 0u;
    }
    // counts member i with key `key`; returns (bucket << 16) | arrival rank
    __device__ uint32_t count(int i, uint32_t key, uint32_t bits) const
    {
        keys[i] = key;
        const uint32_t b = __builtin_amdgcn_ubfe(key, (32u - bits) & 31u, bits);
        const uint32_t sh = (b & 1u) << 4;
        const uint32_t old = atomicAdd(&cnt[b >> 1], 1u << sh);
        return (b << 16) | ((old >> sh) & 0xFFFFu);
    }
};

__device__ __forceinline__ uint32_t sort_bits(int n)
{
    return n >= 2 ? 32u - (uint32_t)__clz(n - 1) : 0u;
}

// After counting (and a barrier): pos[k] of member i = threadIdx.x + k T goes
// from (bucket << 16 | arrival) to the member's position in (key, pid)
// order.  Ends with a barrier.
template <int T, int K, int CAP>
__device__ void rank_in_lds(uint32_t (&pos)[K], int n, uint32_t bits, const SortLDS<T, CAP> &L,
                            const uint32_t *pid_c, uint32_t *wtot)
{
    constexpr int PERW = SortLDS<T, CAP>::PERW;
    const uint32_t nbk = 1u << bits;
    {
        // exclusive scan of the bucket counts over the per-thread chunks
        uint32_t *own = L.own();
        uint32_t c[PERW], s = 0;
#pragma unroll
        for (int q = 0; q < PERW; ++q) {
            c[q] = own[q];
            s += (c[q] & 0xFFFFu) + (c[q] >> 16);
        }
        uint32_t run = block_excl(s, wtot);
#pragma unroll
        for (int q = 0; q < PERW; ++q) {
            const uint32_t lo16 = run, hi16 = run + (c[q] & 0xFFFFu);
            run = hi16 + (c[q] >> 16);
            own[q] = lo16 | (hi16 << 16);
        }
    }
    __syncthreads();
    // keys and members in bucket order
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = threadIdx.x + k * T;
        if (i < n) {
            const uint32_t slot = get16(L.cnt, pos[k] >> 16) + (pos[k] & 0xFFFFu);
            L.sk[slot] = L.keys[i];
            L.lst[slot] = (uint16_t)i;
        }
    }
    __syncthreads();
    // position = bucket start + rank by (key, pid) inside the bucket; the
    // first four members are compared without a loop
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = threadIdx.x + k * T;
        if (i < n) {
            const uint32_t b = pos[k] >> 16, arr = pos[k] & 0xFFFFu;
            const uint32_t beg = get16(L.cnt, b);
            const uint32_t size = ((b + 1 < nbk) ? get16(L.cnt, b + 1) : (uint32_t)n) - beg;
            const uint32_t *skb = L.sk + beg;
            const uint32_t key = skb[arr];
            uint32_t r = 0, tie = 0;
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j) {
                const uint32_t kj = skb[j];
                const bool in = j < size;
                r += (in && kj < key) ? 1u : 0u;
                tie |= (in && kj == key && j != arr) ? 1u : 0u;
            }
            for (uint32_t j = 4; j < size; ++j) {
                const uint32_t kj = skb[j];
                r += kj < key ? 1u : 0u;
                tie |= (kj == key && j != arr) ? 1u : 0u;
            }
            if (tie) {
                // equal keys: the smaller pid comes first
                const uint32_t pi = pid_c[i];
                for (uint32_t j = 0; j < size; ++j)
                    if (j != arr && skb[j] == key && pid_c[L.lst[beg + j]] < pi) ++r;
            }
            pos[k] = beg + r;
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Per-particle global scratch for cells handled by one workgroup without the
// LDS capacity limit, indexed by storage slot (regions of different cells
// never overlap).
// ---------------------------------------------------------------------------
struct HugeScratch {
    uint32_t *keys;    // [n] sort keys
    uint32_t *cnt;     // [n] bucket counts, then offsets
    uint32_t *lst;     // [n] bucket member lists, then slots in sorted order
    uint32_t *pos;     // [n] arrival rank, then sorted position
    uint32_t *w23;     // [2n] words 2 and 3 of the particle draw
    uint8_t *cand;     // [n] null-collision candidate flags
    void *pbuf;        // [n/2 + 2] pair records
};
const HugeScratch &huge_scratch();

// Multi-workgroup path for cells beyond the largest LDS class.  A cell's
// members are split into S segments by their sort key: segment
// floor(key S / 2^32), an equal split of the key range.  Since the order is
// by key first, the cell's sorted order is the segments' sorted orders one
// after another.  Each segment (at most the
// segment capacity, seg_cap) is sorted and paired in LDS by its own workgroup at its
// global offset in the cell; the pair that straddles two segments (when a
// segment starts at an odd position) is done by a fix-up pass.  Members are
// first copied segment-major into the scratch below.
constexpr int SEG_CHUNK = 8192;        // members per counting / scatter work item
constexpr int SEG_MAX = 4096;          // at most this many segments per cell
struct SegScratch {
    // per cell of the multi-workgroup list (index h into that list)
    uint32_t *hc_S;       // segment count
    uint8_t *hc_fb;       // 1: cell takes the one-workgroup path instead
    int32_t *hc_seg;      // first segment of the cell
    int32_t *hc_chunk;    // first work item of the cell
    // per segment (DevFlags count[SEG_SLOT] of them)
    int32_t *sg_cell;     // h
    uint32_t *sg_cnt, *sg_start, *sg_cur;
    int32_t *bnd_head;    // scratch slot of the member paired across the lower edge, or -1
    int32_t *bnd_tail;    // ... across the upper edge, or -1
    // per work item (DevFlags count[CHUNK_SLOT] of them)
    int32_t *ch_owner;    // h
    // per member, segment-major
    int32_t *m_orig;      // storage slot
    uint32_t *m_pid;
    void *m_v;            // 3 components, stride m_stride
    int64_t m_stride;
    int64_t seg_max, chunk_max;
};
constexpr int SEG_SLOT = 6, CHUNK_SLOT = 7;    // DevFlags head/count slots
size_t seg_scratch_bytes(int dtype, int64_t n, int32_t n_cells);
// base: seg_scratch_bytes of tables; the member arrays (n entries each, v
// 3 n of the dtype) are lent by the caller (free during the collide pass).
void set_seg_scratch(int dtype, int64_t n, int32_t n_cells, void *base, int32_t *m_orig,
                     uint32_t *m_pid, void *m_v);
const SegScratch &seg_scratch();
// Segment target (mean members) and capacity for a dtype.
int seg_cap(int dtype);
int seg_target(int dtype);

// Sorted positions of the members [lo, lo+n) of one cell by (keys, pid):
// bucket b = (key * nb) >> 32 is monotone in the key, so buckets in order and
// (key, pid) order inside a bucket give the full order.  keys[lo..) must be
// set; on return pos[lo + i] is member i's position and lst[lo + p] the
// member at position p.  One workgroup; contains barriers.
__device__ __forceinline__ void gsort_positions(const HugeScratch &hs, const uint32_t *pid, int lo,
                                                int n, uint32_t *wtot)
{
    const int T = blockDim.x;
    const uint32_t nb = n >= 2 ? (uint32_t)(n / 2) : 1u;
    for (int i = threadIdx.x; i < (int)nb; i += T) hs.cnt[lo + i] = 0u;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += T) {
        const uint32_t b = __umulhi(hs.keys[lo + i], nb);
        hs.pos[lo + i] = atomicAdd(&hs.cnt[lo + b], 1u);
    }
    __syncthreads();
    {
        const int per = ((int)nb + T - 1) / T;
        const int b0 = threadIdx.x * per;
        uint32_t s = 0;
        for (int q = 0; q < per; ++q)
            if (b0 + q < (int)nb) s += hs.cnt[lo + b0 + q];
        uint32_t run = block_excl(s, wtot);
        for (int q = 0; q < per; ++q)
            if (b0 + q < (int)nb) {
                const uint32_t c = hs.cnt[lo + b0 + q];
                hs.cnt[lo + b0 + q] = run;
                run += c;
            }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += T) {
        const uint32_t b = __umulhi(hs.keys[lo + i], nb);
        hs.lst[lo + hs.cnt[lo + b] + hs.pos[lo + i]] = (uint32_t)i;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += T) {
        const uint32_t key = hs.keys[lo + i];
        const uint32_t b = __umulhi(key, nb);
        const uint32_t beg = hs.cnt[lo + b];
        const uint32_t end = (b + 1 < nb) ? hs.cnt[lo + b + 1] : (uint32_t)n;
        uint32_t rank = 0;
        for (uint32_t m = beg; m < end; ++m) {
            const uint32_t j = hs.lst[lo + m];
            const uint32_t kj = hs.keys[lo + j];
            if (kj < key) ++rank;
            else if (kj == key && j != (uint32_t)i && pid[lo + j] < pid[lo + i]) ++rank;
        }
        hs.pos[lo + i] = beg + rank;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += T) hs.lst[lo + hs.pos[lo + i]] = (uint32_t)i;
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Host-side launch interfaces (implemented in the .hip files).
// ---------------------------------------------------------------------------
struct RadixPass {
    const int32_t *key_in;
    int32_t *key_out;
    int n32, n64;
    const uint32_t *p32_in[6];
    uint32_t *p32_out[6];
    const uint64_t *p64_in[3];
    uint64_t *p64_out[3];
    int iota_slot;      // payload slot written with the element index (-1: none)
    int64_t n;
    int shift, bits;
    const int *gate;    // non-null: run only if *gate != 0
};

// Optional timing of selected launches with HIP events on the launch stream
// (enabled by pic_time_kernels; no cost when off).  Slots: 0-3 LDS classes of
// the collide pass, 4 multi-block class, 5 order check, 6 work queue,
// 7 re-binning passes, 8 stand-alone null-collision step, 9 learned gate
// decision, 10 relaxation of the judged cells.
enum { KT_CLASS0 = 0, KT_HUGE = 4, KT_CHECK = 5, KT_QUEUE = 6, KT_SORT = 7, KT_MCC = 8, KT_GATE = 9,
       KT_RELAX = 10, KT_DEFER = 11, KT_MOMENTS = 12, KT_DSMC = 13, KT_P2C = 14, KT_RECOMB = 15, KT_NANBU = 16, KT_TRIPLET = 17, KT_WEIGHTED = 18, KT_ALL = 19, KT_SLOTS = 20 };
void ktime_begin(int slot, hipStream_t st);
void ktime_end(int slot, hipStream_t st);
bool ktime_pause();            // returns whether timing was on
void ktime_resume(bool was);

struct BinScratch {
    uint32_t *hist;     // (1 << bits) * nblocks
    uint32_t *bsum;     // scan block sums
};

size_t radix_scratch_bytes(int64_t n);
int radix_pass(const RadixPass &p, const BinScratch &s, hipStream_t st);

// Checks the order of cell_of and writes cell_start as if it were sorted.
// set_unsorted: 0 = only range checks, 1 = raise flags->unsorted on a
// descent, 2 = also latch sticky_state (caller asserted sorted storage).
int launch_bin_check(const int32_t *cell_of, int64_t n, int32_t n_cells, int32_t *cell_start,
                     DevFlags *flags, int set_unsorted, const int *gate, hipStream_t st);
int launch_reset_flags(DevFlags *flags, hipStream_t st);
// Latches sticky_nonfinite when any of the 3 n velocities is not finite.
int launch_check_finite(int dtype, const void *v, int64_t n, DevFlags *flags, hipStream_t st);
// Latches sticky_state when work list `list` is not empty.
int launch_reject_list(DevFlags *flags, int list, hipStream_t st);
int launch_set_step(uint64_t *step_dev, uint64_t value, hipStream_t st);
int launch_step_inc(uint64_t *step_dev, hipStream_t st);
int launch_copy32(uint32_t *dst, const uint32_t *src, int64_t n, const int *gate, hipStream_t st);

// Work queue of cells by size class.
struct ClassCaps {
    int ncls;            // number of LDS classes (<= 4), class ncls = multi-block
    int cap[4];          // max members per cell routed to each class (<= its capacity)
    int blocks_per_cu[5];  // persistent workgroups per CU of classes 0-3 and the multi-block class
    int unified;         // plain steps: the collide pass as one persistent launch
    int wave;            // ... with class 0 on one wave per cell (else on whole workgroups)
};
// lists holds QUEUE_LISTS runs of n_cells entries: the classes, the
// multi-block class at index ncls, and the cells the gate defers at
// LIST_DEFERRED.  With skip (nullable) a deferred cell enters no class; it
// is listed as deferred when visit is set (its null collisions still touch
// it), else left out.
constexpr int LIST_DEFERRED = 5;
constexpr int QUEUE_LISTS = 6;
// With seg (nullable) the cells of the multi-workgroup list are also planned
// into segments (see SegScratch; target members per segment).
int launch_build_queue(const int32_t *cell_start, int32_t n_cells, const ClassCaps &caps,
                       int32_t *lists, DevFlags *flags, const uint8_t *skip, int visit,
                       const SegScratch *seg, int seg_target, hipStream_t st);

struct CollideArgs {
    void *v;               // SoA base
    const void *w;         // per-particle weights of the velocity dtype (variable-weight step), or null
    int64_t n;             // stride between components
    const uint32_t *pid;
    const int32_t *cell_start;
    const double *density;
    const double *dt_scale;  // per-cell dt multiplier (nullable)
    double dt, lnL;
    uint64_t seed, step;
    const uint64_t *step_dev;  // nullable: step read from device memory
    uint32_t flags;
    uint64_t mcc_thr;      // candidate iff word1 < mcc_thr (0 = no null collisions)
    double mass_ratio;
    double *moments;       // PIC_MOMENTS output (M x 14)
    double *debt;          // PIC_CONSERVE_FIX: per-cell shortfall (M x 4) carried between steps
    DevFlags *dflags;
    // pairing export
    int32_t *sorted_out, *partner_out;
    int32_t *order;        // n_cells entries of scratch for the one-launch pass (nullable: class launches)
    int variant;           // pair operator: VAR_TA (the step), VAR_NANBU, VAR_TRIPLET
};
enum { VAR_TA = 0, VAR_NANBU = 1, VAR_TRIPLET = 2 };

// seg_path: the cells beyond the LDS classes were planned into segments by
// the queue builder (only for steps without PIC_CONSERVE_FIX and PIC_MOMENTS).
// live: bit c (classes 0..3, 4 = beyond the LDS classes) clear when the
// caller knows that list is empty; its kernels are then not launched.
int launch_collide(int dtype, const CollideArgs &a, const int32_t *lists, int32_t n_cells,
                   const ClassCaps &caps, int pairs_only, int num_cu, hipStream_t st,
                   bool seg_path = false, uint32_t live = ~0u);
// Null collisions of the deferred list: see k_deferred.
int launch_deferred(int dtype, const CollideArgs &a, const int32_t *lists, int32_t n_cells,
                    int num_cu, hipStream_t st);
ClassCaps collide_caps(int dtype, size_t lds_per_block);
// Largest binary64 class of the plain step when its lean pass takes it (the
// caps of such steps are widened to it; other binary64 steps keep cap[3]).
int lean64_cap();
// Global scratch of the multi-block ("huge") class, indexed by particle slot.
size_t huge_scratch_bytes(int dtype, int64_t n);
void set_huge_scratch(int dtype, int64_t n, void *base);

// ---------------------------------------------------------------- learned gate
struct DevGate {
    unsigned long long steps, skipped, collided, judged, judged_want, false_skip;
    int disabled, have_moments;
    unsigned int judge_count;
    int mom_now;      // this step refreshes the moment sums
    unsigned int pad[6];
};

struct GateArgs {
    const double *moments;   // M x 14 post-step sums of the previous step
    const float *params;     // 4801 binary32 master parameters
    int32_t M;
    float thr;               // skip when the network's probability exceeds thr
    int32_t kmax;            // at most kmax deferred steps in a row
    uint64_t judge_thr;      // judged iff word0 of the cell's domain-2 draw < judge_thr
    int bf16;
    uint64_t seed, step;
    const uint64_t *step_dev;
    int32_t *k_acc;
    uint8_t *skip;
    double *dt_scale;
    uint8_t *want;
    float *prob;
    int32_t *judge_list;
    DevGate *g;
    // analytic moment gate (instead of the network): skip when the estimated
    // relaxation over the tolerance is below thr
    int analytic, replicas;
    double dt, lnL, tol;
    const double *density;   // per cell, nullable (1)
};

struct RelaxArgs {
    const void *v;
    int64_t n;
    const int32_t *cell_start;
    const uint32_t *pid;
    const double *density;
    const double *dt_scale;
    double dt, lnL;
    uint64_t seed, step;
    const uint64_t *step_dev;
    int replicas;
    const int32_t *list;        // cells to evaluate (NULL: cells 0..count-1)
    const uint32_t *count_dev;  // device count of list entries (NULL: count)
    int32_t count;
    double *r_out;              // indexed by cell
    const DevFlags *dflags;     // in a collision step: skip when binning failed
    int assume_sorted;
    double *part;               // scratch of relax_part_bytes(cap, replicas) bytes
    int32_t cap;                // most entries the list can hold (scratch sizing)
    // set by launch_relax inside the scratch: list positions by size class
    // (3 runs of cap) and the class counts
    int32_t *cls_list;
    uint32_t *cls_count;
};
// Scratch bytes of launch_relax for lists of up to `count` cells: the
// per-replica tensor sums [count * replicas * 6] and the size-class lists.
size_t relax_part_bytes(int64_t count, int replicas);

int launch_features(const double *moments, int32_t M, float *feat, uint8_t *valid, hipStream_t st);
int launch_mlp_forward(const float *params, const float *x, int32_t B, int bf16, float *prob,
                       hipStream_t st);
int launch_gate_infer_decide(const float *prob, int32_t M, float thr, int32_t kmax, uint8_t *skip,
                             int32_t *k_acc, hipStream_t st);
size_t mlp_grad_scratch_floats(int32_t B);
int launch_mlp_grad(const float *params, const float *x, const float *y, int32_t B, int bf16,
                    float *scratch, float *grad, float *loss, hipStream_t st);
int launch_adam(float *params, float *m, float *v, const float *grad, int32_t t, float lr,
                hipStream_t st);
int launch_gate(const GateArgs &a, hipStream_t st);
int launch_analytic_relax(const double *moments, int32_t M, double dt, double lnL, const double *density,
                          int replicas, double *r, hipStream_t st);
int launch_gate_score(DevGate *g, const int32_t *judge_list, const uint8_t *want, const double *r,
                      double tol, double max_false, uint32_t min_judged, hipStream_t st);
int launch_relax(int dtype, const RelaxArgs &a, int num_cu, hipStream_t st);
int launch_gate_end(DevGate *g, hipStream_t st);
// Sets g->mom_now for this step (before the collide launches).
int launch_mom_select(DevGate *g, const uint64_t *step_dev, uint64_t step, int every,
                      hipStream_t st);

// Exact-count selection: the k particles with the smallest candidate words
// ((pid, slot) breaks ties) scatter.  ws: mcc_exact_ws_bytes(n, k) of scratch.
size_t mcc_exact_ws_bytes(int64_t n, int64_t k);
int launch_mcc_exact(int dtype, void *v, const uint32_t *pid, int64_t n, int64_t k, double mass_ratio,
                     uint64_t seed, uint64_t step, uint8_t *selected_out, void *ws, hipStream_t st);
int launch_mcc(int dtype, void *v, const uint32_t *pid, int64_t n, uint64_t thr, double mass_ratio,
               uint64_t seed, uint64_t step, uint8_t *cand_out, hipStream_t st);
int launch_philox(uint64_t seed, uint64_t step, uint32_t domain, uint32_t c3, const uint32_t *c0,
                  int64_t n, uint32_t *out, hipStream_t st);
// Per-cell moment sums (layout of pic_cell_moments); with run_if (nullable)
// the pass runs only when *run_if is nonzero.
// Electron-heavy collision channels C1..C4 (see dsmc_collide).
constexpr int DSMC_MAX_SEG = 64;
struct DsmcTable {
    int32_t nseg;
    const double *breaks;   // device [nseg + 1]
    const double *coef;     // device [4][nseg][4]
    double thr[4];
    double mass_ratio;
};
struct DsmcArgs {
    void *v;
    int64_t n;
    int32_t n_cells;
    const int32_t *cell;
    const uint32_t *pid;
    const double *ng, *nm;  // per-cell densities (nullable)
    double ng0, nm0, dt;
    uint64_t seed, step;
    uint32_t pid_base;
    void *v_new;
    int64_t cap;
    uint32_t *pid_new;
    int32_t *cell_new;
    unsigned long long *count;
    uint8_t *chan_out;
    DevFlags *dflags;
};
int launch_dsmc(int dtype, const DsmcArgs &a, const DsmcTable &t, hipStream_t st);

// Recombination C5 on cell-sorted storage (v and w of the velocity dtype).
struct RecombArgs {
    void *v;
    void *w;
    const uint32_t *pid;
    const uint8_t *primary;
    int64_t n;
    const int32_t *cs;
    int32_t M;
    double eps;
    uint64_t seed;
    uint32_t step;
    int32_t *events;
};
int launch_recombine(int dtype, const RecombArgs &a, int num_cu, hipStream_t st);

// Particle-to-cell sums out[j * nq + k] (binary64) of nq <= 4 quantities
// q[k * n + l] over the particles l of cell j.  ws: p2c_ws_bytes(...).
size_t p2c_ws_bytes(int64_t n, int32_t M, int nq, int num_cu);
int launch_p2c(int dtype, int nq, const void *q, const int32_t *cell_of, int64_t n, int32_t M, double *out,
               void *ws, DevFlags *f, int num_cu, hipStream_t st);

int launch_moments(int dtype, const void *v, int64_t n, const int32_t *cell_start,
                   int32_t n_cells, double *out, const int *run_if, int num_cu, hipStream_t st);
int launch_unsort(int dtype, void *v, uint32_t *pid, int32_t *cell_of, int64_t n, void *tmp,
                  hipStream_t st);

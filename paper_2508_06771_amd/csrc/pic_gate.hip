// pic_gate.hip -- learned sub-cycling gate of the collision step.
//
// A cell whose Coulomb relaxation over one step is below a tolerance can
// defer its collision: it accumulates the skipped time and later collides
// once with dt_eff = (k + 1) dt.  A small network decides from eight moment
// features per cell; the plain operator stays the fallback and, on a
// Philox-sampled fraction of cells every step, the judge of the network's
// decisions.
//
//   features   eight Galilean-invariant moments of the cell from its 14 FP64
//              raw sums (count, momentum, second moments, heat flux, |v|^4)
//   network    8 -> 64 -> 64 -> 1, ReLU, logistic output; BF16 products with
//              FP32 accumulation (or FP32 throughout), FP32 master weights
//   label      expected relative one-step change of the temperature tensor,
//              r = || E sum_pairs 1/4 h(s^2) (|u|^2 I - 3 u u^T) || / (N T),
//              averaged over independent re-pairings; h(s^2) = E[sin^2 Theta]
//   training   forward, binary cross-entropy, backward and Adam, all here
#include "pic_internal.hpp"

#define HIP_OK(x) do { if ((x) != hipSuccess) return PIC_ERR_HIP; } while (0)

namespace {

constexpr double PI_D = 3.14159265358979323846;
constexpr int OFF_W1 = 0, OFF_B1 = 512, OFF_W2 = 576, OFF_B2 = 4672, OFF_W3 = 4736, OFF_B3 = 4800;
constexpr int NPARAM = 4801;

// Round a binary32 value to bfloat16 (nearest, ties to even), returned as binary32.
__device__ __forceinline__ float bf16r(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xFFFF0000u);
}

// h(s^2) = E[sin^2 Theta] = E[4 d^2 / (1 + d^2)^2], d ~ N(0, s^2).  With
// E[1/(1 + t z^2)] = sqrt(pi/(2t)) erfcx(1/sqrt(2t)) and h = -4 t d/dt of it:
// h = 2 sqrt(pi) w (1 + 2 w^2) erfcx(w) - 4 w^2, w = 1 / sqrt(2 t).  Below
// t = 1e-3 the closed form cancels (relative error ~1e-16 / t), so the
// asymptotic Gaussian-moment series is used there (next term ~ 2.5e5 t^6,
// below 1e-10 relative).
__device__ __noinline__ double h_angle(double t)
{
    if (t < 1e-3) {
        return t * (4.0 + t * (-24.0 + t * (180.0 + t * (-1680.0 + t * 18900.0))));
    }
    const double w = 1.0 / sqrt(2.0 * t);
    return 2.0 * sqrt(PI_D) * w * (1.0 + 2.0 * w * w) * erfcx(w) - 4.0 * w * w;
}

// Eight features from the raw sums m[0..13] (layout of pic_cell_moments).
// Returns false for cells with fewer than two members or no temperature.
__device__ bool features_from_sums(const double *m, float f[8])
{
    const double N = m[0];
    for (int k = 0; k < 8; ++k) f[k] = 0.0f;
    if (!(N >= 2.0)) return false;
    const double V[3] = {m[1] / N, m[2] / N, m[3] / N};
    const double Q = m[4] + m[5] + m[6];   // sum |v|^2
    // central second moments T_ab = <v_a v_b> - V_a V_b
    const double Txx = m[4] / N - V[0] * V[0], Tyy = m[5] / N - V[1] * V[1], Tzz = m[6] / N - V[2] * V[2];
    const double Txy = m[7] / N - V[0] * V[1], Txz = m[8] / N - V[0] * V[2], Tyz = m[9] / N - V[1] * V[2];
    const double T = (Txx + Tyy + Tzz) / 3.0;
    if (!(T > 0.0)) return false;
    const double S2[3][3] = {{m[4], m[7], m[8]}, {m[7], m[5], m[9]}, {m[8], m[9], m[6]}};
    const double VV = V[0] * V[0] + V[1] * V[1] + V[2] * V[2];
    // sum |c|^2 c_a = S3_a - V_a Q - 2 (S2 V)_a + 2 V_a N |V|^2
    double q[3];
    for (int a = 0; a < 3; ++a) {
        const double s2v = S2[a][0] * V[0] + S2[a][1] * V[1] + S2[a][2] * V[2];
        q[a] = 0.5 * (m[10 + a] - V[a] * Q - 2.0 * s2v + 2.0 * V[a] * N * VV);
    }
    // sum |c|^4 = S4 - 4 V.S3 + 4 V^T S2 V + 2 |V|^2 Q - 3 N |V|^4
    double vs2v = 0.0;
    for (int a = 0; a < 3; ++a)
        vs2v += V[a] * (S2[a][0] * V[0] + S2[a][1] * V[1] + S2[a][2] * V[2]);
    const double c4 = m[13] - 4.0 * (V[0] * m[10] + V[1] * m[11] + V[2] * m[12]) + 4.0 * vs2v +
                      2.0 * VV * Q - 3.0 * N * VV * VV;
    f[0] = (float)log(N);
    f[1] = (float)log(T);
    // diagonal anisotropy centred on isotropy (computed before rounding, so
    // bfloat16 inputs keep the resolution of small anisotropies)
    f[2] = (float)((Txx - T) / T);
    f[3] = (float)((Tyy - T) / T);
    f[4] = (float)((Tzz - T) / T);
    f[5] = (float)(sqrt(2.0 * (Txy * Txy + Txz * Txz + Tyz * Tyz)) / T);
    f[6] = (float)(sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]) / (N * T * sqrt(T)));
    f[7] = (float)(c4 / N / (15.0 * T * T) - 1.0);
    return true;
}

// Network logit of one sample; P holds the parameters (weights already
// rounded to bfloat16 in BF16 mode), products of bfloat16-rounded operands,
// binary32 accumulation.
__device__ float mlp_logit(const float *P, const float x_in[8], bool bf16)
{
    float x[8];
    for (int i = 0; i < 8; ++i) x[i] = bf16 ? bf16r(x_in[i]) : x_in[i];
    float h1[64];
    for (int j = 0; j < 64; ++j) {
        float z = P[OFF_B1 + j];
        for (int i = 0; i < 8; ++i) z += x[i] * P[OFF_W1 + i * 64 + j];
        z = z > 0.0f ? z : 0.0f;
        h1[j] = bf16 ? bf16r(z) : z;
    }
    float out = P[OFF_B3];
    for (int j = 0; j < 64; ++j) {
        float z = P[OFF_B2 + j];
        for (int i = 0; i < 64; ++i) z += h1[i] * P[OFF_W2 + i * 64 + j];
        z = z > 0.0f ? z : 0.0f;
        out += (bf16 ? bf16r(z) : z) * P[OFF_W3 + j];
    }
    return out;
}

__device__ void load_params(float *P, const float *params, bool bf16)
{
    for (int p = threadIdx.x; p < NPARAM; p += blockDim.x) {
        const bool weight = p < OFF_B1 || (p >= OFF_W2 && p < OFF_B2) || (p >= OFF_W3 && p < OFF_B3);
        P[p] = (bf16 && weight) ? bf16r(params[p]) : params[p];
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_features(const double *__restrict__ mom, int32_t M,
                                                  float *__restrict__ feat, uint8_t *__restrict__ valid)
{
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < M; j += gridDim.x * blockDim.x) {
        float f[8];
        const bool ok = features_from_sums(mom + (int64_t)j * 14, f);
        for (int k = 0; k < 8; ++k) feat[(int64_t)j * 8 + k] = f[k];
        if (valid) valid[j] = ok;
    }
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float *__restrict__ params,
                                                     const float *__restrict__ x, int32_t B, int bf16,
                                                     float *__restrict__ prob)
{
    __shared__ float P[NPARAM];
    load_params(P, params, bf16 != 0);
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < B; s += gridDim.x * blockDim.x) {
        float xi[8];
        for (int i = 0; i < 8; ++i) xi[i] = x[(int64_t)s * 8 + i];
        const float z = mlp_logit(P, xi, bf16 != 0);
        prob[s] = 1.0f / (1.0f + __expf(-z));
    }
}

// ------------------------------------------------------------ matrix-core network
// bfloat16 mode on the matrix cores: one wave evaluates 32 samples with
// v_mfma_f32_32x32x8_bf16 (A 32x8 rows x k, B 8x32 k x columns, FP32
// accumulation).  Operand layout of that instruction: A[i][k] sits in lane
// i + 32 (k / 4), element k % 4; B[k][j] in lane j + 32 (k / 4), element
// k % 4; D[i][j] in lane j + 32 ((i / 4) % 2), element 4 (i / 8) + i % 4.
// Layer 1 is one product per 32 output columns; the hidden layer goes
// through LDS to change from the D to the A layout; layer 2 is eight
// products of k = 8 per 32 columns; the output layer is a lane reduction.
// The rounding points are those of mlp_logit: bfloat16 inputs, weights and
// hidden activations, binary32 sums (here in the matrix core's order).
typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

__device__ __forceinline__ short bf16_bits(float x)
{
    return (short)(__float_as_uint(bf16r(x)) >> 16);
}

constexpr int MLP_ROW = 64 + 4;   // padded LDS rows (bank spread)

struct __align__(16) MlpLDS {
    short w1t[64][8];           // W1 transposed, [column][k], bfloat16
    short w2t[64][MLP_ROW];     // W2 transposed, [column][k], bfloat16
    float b1[64], b2[64], w3[64], b3;
};

struct __align__(16) MlpWave {
    short h1[32][MLP_ROW];      // hidden layer 1 of the wave's 32 samples
};

__device__ void load_mlp_lds(MlpLDS &P, const float *params)
{
    for (int p = threadIdx.x; p < 8 * 64; p += blockDim.x) {
        const int i = p / 64, j = p % 64;
        P.w1t[j][i] = bf16_bits(params[OFF_W1 + p]);
    }
    for (int p = threadIdx.x; p < 64 * 64; p += blockDim.x) {
        const int i = p / 64, j = p % 64;
        P.w2t[j][i] = bf16_bits(params[OFF_W2 + p]);
    }
    for (int j = threadIdx.x; j < 64; j += blockDim.x) {
        P.b1[j] = params[OFF_B1 + j];
        P.b2[j] = params[OFF_B2 + j];
        P.w3[j] = bf16r(params[OFF_W3 + j]);
    }
    if (threadIdx.x == 0) P.b3 = params[OFF_B3];
}

__device__ __forceinline__ void wave_lds_order()
{
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// Logit of sample (lane % 32) of the wave's 32; x: that sample's features
// (both half-waves hold them).  Every lane of the wave must take part.
__device__ float mlp_logit_mfma(const MlpLDS &P, const float x[8], MlpWave &W)
{
    const int lane = threadIdx.x & (PIC_WAVE - 1);
    const int half = lane >> 5, c = lane & 31;
    bf16x4_t a, b0, b1;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        a[j] = bf16_bits(half ? x[4 + j] : x[j]);
        b0[j] = P.w1t[c][4 * half + j];
        b1[j] = P.w1t[c + 32][4 * half + j];
    }
    f32x16_t d0, d1;
#pragma unroll
    for (int r = 0; r < 16; ++r) d0[r] = d1[r] = 0.0f;
    d0 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b0, d0, 0, 0, 0);
    d1 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b1, d1, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = 8 * (r / 4) + 4 * half + (r % 4);
        const float z0 = d0[r] + P.b1[c], z1 = d1[r] + P.b1[c + 32];
        W.h1[row][c] = bf16_bits(z0 > 0.0f ? z0 : 0.0f);
        W.h1[row][c + 32] = bf16_bits(z1 > 0.0f ? z1 : 0.0f);
    }
    wave_lds_order();
    f32x16_t e0, e1;
#pragma unroll
    for (int r = 0; r < 16; ++r) e0[r] = e1[r] = 0.0f;
#pragma unroll
    for (int kc = 0; kc < 8; ++kc) {
        const bf16x4_t ah = *(const bf16x4_t *)&W.h1[c][8 * kc + 4 * half];
        const bf16x4_t w0 = *(const bf16x4_t *)&P.w2t[c][8 * kc + 4 * half];
        const bf16x4_t w1 = *(const bf16x4_t *)&P.w2t[c + 32][8 * kc + 4 * half];
        e0 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah, w0, e0, 0, 0, 0);
        e1 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah, w1, e1, 0, 0, 0);
    }
    float sum[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const float z0 = e0[r] + P.b2[c], z1 = e1[r] + P.b2[c + 32];
        sum[r] = bf16r(z0 > 0.0f ? z0 : 0.0f) * P.w3[c] + bf16r(z1 > 0.0f ? z1 : 0.0f) * P.w3[c + 32];
    }
#pragma unroll
    for (int r = 0; r < 16; ++r)
#pragma unroll
        for (int o = 16; o >= 1; o >>= 1) sum[r] += __shfl_xor(sum[r], o, 32);
    // every lane of a half-wave now holds the 16 row sums of rows
    // 8 (r / 4) + 4 half + r % 4; sample c's row is among them when
    // bit 2 of c equals half, else the other half-wave holds it
    const int rc = 4 * (c / 8) + (c % 4);
    float mine = sum[0];
#pragma unroll
    for (int r = 1; r < 16; ++r) mine = (rc == r) ? sum[r] : mine;
    const float other = __shfl_xor(mine, 32, PIC_WAVE);
    wave_lds_order();   // the next tile rewrites W
    return (((c >> 2) & 1) == half ? mine : other) + P.b3;
}

__global__ __launch_bounds__(256) void k_mlp_forward_mfma(const float *__restrict__ params,
                                                          const float *__restrict__ x, int32_t B,
                                                          float *__restrict__ prob)
{
    __shared__ MlpLDS P;
    __shared__ MlpWave Wv[4];
    load_mlp_lds(P, params);
    __syncthreads();
    const int wid = threadIdx.x / PIC_WAVE, c = threadIdx.x & 31;
    const int ntiles = (B + 31) / 32;
    for (int tile = blockIdx.x * 4 + wid; tile < ntiles; tile += gridDim.x * 4) {
        const int s = tile * 32 + c;
        float xi[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) xi[i] = s < B ? x[(int64_t)s * 8 + i] : 0.0f;
        const float z = mlp_logit_mfma(P, xi, Wv[wid]);
        if ((threadIdx.x & 32) == 0 && s < B) prob[s] = 1.0f / (1.0f + __expf(-z));
        __builtin_amdgcn_wave_barrier();   // the next tile needs the whole wave
    }
}

// ------------------------------------------------------------ analytic gate
// Estimate of the judged relaxation r (expected one-step change of the
// temperature tensor, averaged over K re-pairings, over N T) from the raw
// moment sums alone, for the gate that needs no network:
//   r^2 = r_aniso^2 + r_floor^2,
//   r_aniso = 3 nu_0 dt ||A||_F: the traceless part A of the temperature
//     tensor (in units of T = tr / 3) decays at 3 nu_0 near isotropy (the
//     bi-Maxwellian T_par - T_perp decays at 3 nu_T), with
//     nu_0 = (8 sqrt(pi) / 15) n lnL / T^1.5, the small-anisotropy limit of
//     the isotropisation rate;
//   r_floor^2 = (c / T^1.5)^2 / N (a - b + (3/2 - a) / K), c = 8 pi n lnL dt:
//     the spread of the pair sum for an isotropic Maxwellian cell with small
//     angles (a pair adds c (I - 3 u^ u^T) / |u|, E|u|^-2 = 1 / (2T)).  Its
//     part that does not depend on the pairing is sum_a g(v_a),
//     g(v) = -psi(|v|) (I - 3 v^ v^T), psi = G'/v - G'' for the Rosenbluth
//     potential G of the Maxwellian, of variance a = 6 E[psi^2] per member
//     (numerical integral over the unit Maxwellian); b = 10 / (25 pi) of it
//     is the sample's second-moment anisotropy already counted in r_aniso.
//     The pairing part (3/2 - a) is divided by K.
// NaN for cells of fewer than two members or no temperature.
constexpr double ANALYTIC_A = 0.15215976481548635;   // 6 E[psi^2]
constexpr double ANALYTIC_B = 10.0 / (25.0 * PI_D);

__device__ double analytic_relax(const double *m, double dt, double lnL, double n, int K)
{
    const double N = m[0];
    if (!(N >= 2.0)) return __longlong_as_double(0x7ff8000000000000ll);
    const double Vx = m[1] / N, Vy = m[2] / N, Vz = m[3] / N;
    const double Txx = m[4] / N - Vx * Vx, Tyy = m[5] / N - Vy * Vy, Tzz = m[6] / N - Vz * Vz;
    const double Txy = m[7] / N - Vx * Vy, Txz = m[8] / N - Vx * Vz, Tyz = m[9] / N - Vy * Vz;
    const double T = (Txx + Tyy + Tzz) / 3.0;
    if (!(T > 0.0)) return __longlong_as_double(0x7ff8000000000000ll);
    const double a2 = ((Txx - T) * (Txx - T) + (Tyy - T) * (Tyy - T) + (Tzz - T) * (Tzz - T) +
                       2.0 * (Txy * Txy + Txz * Txz + Tyz * Tyz)) / (T * T);
    const double t15 = T * sqrt(T);
    const double r_aniso = 8.0 * sqrt(PI_D) / 5.0 * n * lnL * dt * sqrt(a2) / t15;
    const double c = 8.0 * PI_D * n * lnL * dt / t15;
    const double floor2 = c * c / N * (ANALYTIC_A - ANALYTIC_B + (1.5 - ANALYTIC_A) / (double)K);
    return sqrt(r_aniso * r_aniso + floor2);
}

__global__ __launch_bounds__(256) void k_analytic_relax(const double *__restrict__ mom, int32_t M, double dt,
                                                        double lnL, const double *__restrict__ density,
                                                        int K, double *__restrict__ r)
{
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < M; j += gridDim.x * blockDim.x)
        r[j] = analytic_relax(mom + (int64_t)j * 14, dt, lnL, density ? density[j] : 1.0, K);
}

// ------------------------------------------------------------ gate per step
// Decision for cell j from the network's probability p, or in the analytic
// gate from p = estimated relaxation / tolerance (valid: the cell has
// features and the gate is on).
__device__ __forceinline__ void gate_decide(const GateArgs &a, int j, bool valid, float p, uint64_t step,
                                            bool on, bool judge_now)
{
    const bool pass = a.analytic ? p < a.thr : p > a.thr;
    const bool want = valid && pass && a.k_acc[j] < a.kmax;
    const W4 w = draw4(a.seed, (uint32_t)j, (uint32_t)step, 2u, 0u);
    const bool judge = on && judge_now && (uint64_t)w.x < a.judge_thr;
    const bool skip = want && !judge;
    a.prob[j] = valid ? p : 0.0f;
    a.want[j] = (uint8_t)((want ? 1u : 0u) | (judge ? 2u : 0u));   // bit 1: judged
    a.skip[j] = skip;
    if (skip) {
        a.k_acc[j] += 1;
        a.dt_scale[j] = 0.0;
    } else {
        a.dt_scale[j] = (double)(a.k_acc[j] + 1);
        a.k_acc[j] = 0;
    }
}

// One workgroup: the judged cells in ascending order (from bit 1 of want),
// their count, and the step's skipped / collided totals.  No atomics: the
// decision kernel writes flags only (contended counters across the chip's
// L2 slices cost more than the network itself).
__global__ __launch_bounds__(1024) void k_gate_list(DevGate *g, const uint8_t *__restrict__ want,
                                                    const uint8_t *__restrict__ skip, int32_t M,
                                                    int32_t *__restrict__ judge_list)
{
    __shared__ uint32_t wtot[16];
    // each thread owns a contiguous run of 16-cell words (16-byte loads; the
    // flag arrays are 256-byte aligned and padded, reads past M are masked)
    const int words = (M + 15) / 16;
    const int per = (words + (int)blockDim.x - 1) / (int)blockDim.x;
    const int w0 = (int)threadIdx.x * per;
    const uint4 *wv = (const uint4 *)want, *sv = (const uint4 *)skip;
    uint32_t nj = 0, ns = 0;
    for (int q = 0; q < per; ++q) {
        const int w = w0 + q;
        if (w < words) {
            const uint4 a = wv[w], b = sv[w];
            const uint32_t aw[4] = {a.x, a.y, a.z, a.w}, bw[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                if (w * 16 + e < M) {
                    nj += (aw[e / 4] >> (8 * (e % 4) + 1)) & 1u;
                    ns += (bw[e / 4] >> (8 * (e % 4))) & 1u;
                }
            }
        }
    }
    uint32_t off = block_excl(nj, wtot);
    const uint32_t sk_before = block_excl(ns, wtot);
    if (nj) {
        for (int q = 0; q < per; ++q) {
            const int w = w0 + q;
            if (w < words) {
                const uint4 a = wv[w];
                const uint32_t aw[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    if (w * 16 + e < M && ((aw[e / 4] >> (8 * (e % 4) + 1)) & 1u)) judge_list[off++] = w * 16 + e;
            }
        }
    }
    if (threadIdx.x == blockDim.x - 1) {
        const uint32_t skipped = sk_before + ns;
        g->judge_count = off;
        g->skipped += skipped;
        g->collided += (unsigned long long)M - skipped;
    }
}

// One thread per cell (binary32 network): decide skip / collide, with the
// deferred-time count.
__global__ __launch_bounds__(256) void k_gate(GateArgs a)
{
    __shared__ float P[NPARAM];
    load_params(P, a.params, false);
    const uint64_t step = a.step_dev ? *a.step_dev : a.step;
    const bool on = a.g->have_moments && !a.g->disabled;
    const bool judge_now = a.g->mom_now != 0;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < a.M; j += gridDim.x * blockDim.x) {
        float p = 0.0f;
        bool valid = false;
        if (on) {
            float f[8];
            valid = features_from_sums(a.moments + (int64_t)j * 14, f);
            if (valid) p = 1.0f / (1.0f + __expf(-mlp_logit(P, f, false)));
        }
        gate_decide(a, j, valid, p, step, on, judge_now);
    }
}

// The analytic gate: one thread per cell, the estimate in binary64.
__global__ __launch_bounds__(256) void k_gate_analytic(GateArgs a)
{
    const uint64_t step = a.step_dev ? *a.step_dev : a.step;
    const bool on = a.g->have_moments && !a.g->disabled;
    const bool judge_now = a.g->mom_now != 0;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < a.M; j += gridDim.x * blockDim.x) {
        float q = 0.0f;
        bool valid = false;
        if (on) {
            const double r = analytic_relax(a.moments + (int64_t)j * 14, a.dt, a.lnL,
                                            a.density ? a.density[j] : 1.0, a.replicas);
            valid = r == r;
            if (valid) q = (float)(r / a.tol);
        }
        gate_decide(a, j, valid, q, step, on, judge_now);
    }
}

// The same decision with the bfloat16 network on the matrix cores: one wave
// per 32 cells.
__global__ __launch_bounds__(256) void k_gate_mfma(GateArgs a)
{
    __shared__ MlpLDS P;
    __shared__ MlpWave Wv[4];
    load_mlp_lds(P, a.params);
    __syncthreads();
    const uint64_t step = a.step_dev ? *a.step_dev : a.step;
    const bool on = a.g->have_moments && !a.g->disabled;
    const bool judge_now = a.g->mom_now != 0;
    const int wid = threadIdx.x / PIC_WAVE, c = threadIdx.x & 31;
    const int ntiles = (a.M + 31) / 32;
    for (int tile = blockIdx.x * 4 + wid; tile < ntiles; tile += gridDim.x * 4) {
        const int j = tile * 32 + c;
        float f[8];
        bool valid = false;
        if (on && j < a.M) valid = features_from_sums(a.moments + (int64_t)j * 14, f);
        if (!valid) {
#pragma unroll
            for (int i = 0; i < 8; ++i) f[i] = 0.0f;
        }
        float p = 0.0f;
        if (on) p = 1.0f / (1.0f + __expf(-mlp_logit_mfma(P, f, Wv[wid])));
        if ((threadIdx.x & 32) == 0 && j < a.M) gate_decide(a, j, valid, p, step, on, judge_now);
        __builtin_amdgcn_wave_barrier();   // the next tile needs the whole wave
    }
}

// ------------------------------------------------------------ relaxation label
// The evaluated cells are first split by size (k_relax_classify).  Cells of
// at most RELAX_LDS_CAP members: one workgroup per (cell, replica) sorts the
// replica's keys in LDS and sums the pair terms 1/4 h(s^2) (|u|^2 I - 3 u u^T)
// into part[]; k_relax_finish adds the replicas in order and normalises.
// Larger cells take k_relax below.
constexpr int RELAX_T0 = 256, RELAX_K0 = 8;      // <= 2048 members
constexpr int RELAX_T1 = 1024, RELAX_K1 = 10;    // <= 10240 members
constexpr int RELAX_LDS_CAP = RELAX_T1 * RELAX_K1;
constexpr int RELAX_CLASSIFY_T = 512;            // class counts per pass fit 10 bits

__device__ __forceinline__ bool relax_off(const RelaxArgs &a)
{
    return a.dflags && (a.dflags->range_err || (a.assume_sorted && a.dflags->unsorted));
}

__device__ __forceinline__ int relax_cell(const RelaxArgs &a, uint32_t which)
{
    return a.list ? a.list[which] : (int)which;
}

// One workgroup: positions in the evaluated list by size class (0: LDS sort
// by RELAX_T0 threads, 1: by RELAX_T1 threads, 2: sort in global scratch), in
// ascending order, and the class counts.  The three per-class flags are
// packed into one scan (10 bits each).
__global__ __launch_bounds__(RELAX_CLASSIFY_T) void k_relax_classify(RelaxArgs a)
{
    __shared__ uint32_t wtot[RELAX_CLASSIFY_T / PIC_WAVE];
    __shared__ uint32_t s_tot;
    if (relax_off(a)) return;
    const uint32_t count = a.count_dev ? *a.count_dev : (uint32_t)a.count;
    uint32_t base[3] = {0, 0, 0};
    for (uint32_t c0 = 0; c0 < count; c0 += RELAX_CLASSIFY_T) {
        const uint32_t which = c0 + threadIdx.x;
        int cls = -1;
        if (which < count) {
            const int cell = relax_cell(a, which);
            const int n = a.cell_start[cell + 1] - a.cell_start[cell];
            cls = n <= RELAX_T0 * RELAX_K0 ? 0 : n <= RELAX_LDS_CAP ? 1 : 2;
        }
        const uint32_t flag = cls < 0 ? 0u : 1u << (10 * cls);
        const uint32_t off = block_excl(flag, wtot);
        if (threadIdx.x == RELAX_CLASSIFY_T - 1) s_tot = off + flag;
        __syncthreads();
        const uint32_t tot = s_tot;
        if (cls >= 0) {
            const uint32_t o = (off >> (10 * cls)) & 1023u;
            a.cls_list[(int64_t)cls * a.cap + base[cls] + o] = (int32_t)which;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) base[c] += (tot >> (10 * c)) & 1023u;
        __syncthreads();   // s_tot is rewritten by the next pass
    }
    if (threadIdx.x < 3) a.cls_count[threadIdx.x] = base[threadIdx.x];
}

template <typename R, int T, int K>
__global__ __launch_bounds__(T) void k_relax_lds(RelaxArgs a, int cls)
{
    constexpr int CAP = T * K;
    constexpr int PK = (CAP / 2 + T - 1) / T;    // pairs per thread
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[8 * (T / PIC_WAVE)];
    __shared__ uint32_t wtot[T / PIC_WAVE];
    if (relax_off(a)) return;
    const uint32_t reps = (uint32_t)a.replicas;
    const uint32_t items = a.cls_count[cls] * reps;
    const int32_t *mine = a.cls_list + (int64_t)cls * a.cap;
    const uint32_t step = (uint32_t)(a.step_dev ? *a.step_dev : a.step);
    const SortLDS<T, CAP> L(smem);
    for (uint32_t item = blockIdx.x; item < items; item += gridDim.x) {
        const uint32_t which = (uint32_t)mine[item / reps], rep = item % reps;
        const int cell = relax_cell(a, which);
        const int lo = a.cell_start[cell];
        const int n = a.cell_start[cell + 1] - lo;
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // xx yy zz xy xz yz
        if (n >= 2 && n <= CAP) {
            const uint32_t *pid_c = a.pid + lo;
            const uint32_t bits = sort_bits(n);
            uint32_t pos[K];
            // the pids are loaded before any is used (pos holds them until
            // the keys are counted), so the loads are in flight together
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int i = threadIdx.x + k * T;
                if (i < n) pos[k] = pid_c[i];
            }
            L.clear();
            __syncthreads();
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int i = threadIdx.x + k * T;
                if (i < n) pos[k] = L.count(i, draw4(a.seed, pos[k], step, 3u, rep).x, bits);
            }
            __syncthreads();
            rank_in_lds<T, K, CAP>(pos, n, bits, L, pid_c, wtot);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int i = threadIdx.x + k * T;
                if (i < n) L.lst[pos[k]] = (uint16_t)i;
            }
            __syncthreads();
            const R *vx = (const R *)a.v + lo;
            const R *vy = (const R *)a.v + a.n + lo;
            const R *vz = (const R *)a.v + 2 * a.n + lo;
            const double dens = a.density ? a.density[cell] : 1.0;
            const double dts = a.dt_scale ? a.dt_scale[cell] : 1.0;
            const double C = 8.0 * PI_D * dens * a.lnL * a.dt * dts;
            // all of the thread's pairs are gathered before any is evaluated,
            // so their loads are in flight together
            double ux[PK], uy[PK], uz[PK];
#pragma unroll
            for (int k = 0; k < PK; ++k) {
                const int q = threadIdx.x + k * T;
                ux[k] = uy[k] = uz[k] = 0.0;
                if (q < n / 2) {
                    const int ia = L.lst[2 * q], ib = L.lst[2 * q + 1];
                    ux[k] = (double)vx[ia] - (double)vx[ib];
                    uy[k] = (double)vy[ia] - (double)vy[ib];
                    uz[k] = (double)vz[ia] - (double)vz[ib];
                }
            }
#pragma unroll
            for (int k = 0; k < PK; ++k) {
                const double uu = ux[k] * ux[k] + uy[k] * uy[k] + uz[k] * uz[k];
                if (uu == 0.0) continue;   // also the slots past the last pair
                const double hq = 0.25 * h_angle(C / (uu * sqrt(uu)));
                acc[0] += hq * (uu - 3.0 * ux[k] * ux[k]);
                acc[1] += hq * (uu - 3.0 * uy[k] * uy[k]);
                acc[2] += hq * (uu - 3.0 * uz[k] * uz[k]);
                acc[3] += hq * (-3.0 * ux[k] * uy[k]);
                acc[4] += hq * (-3.0 * ux[k] * uz[k]);
                acc[5] += hq * (-3.0 * uy[k] * uz[k]);
            }
        }
        // its barriers also end this item's use of LDS
        const double t = block_sum_scatter<8>(acc, red);
        if (threadIdx.x < 6) a.part[((size_t)which * reps + rep) * 6 + threadIdx.x] = t;
    }
}

// One workgroup per listed cell of at most RELAX_LDS_CAP members: the cell's
// temperature, the replica sums in replica order, r.
template <typename R>
__global__ __launch_bounds__(256) void k_relax_finish(RelaxArgs a)
{
    __shared__ double red[5 * 4];
    if (a.dflags && (a.dflags->range_err || (a.assume_sorted && a.dflags->unsorted))) return;
    const uint32_t count = a.count_dev ? *a.count_dev : (uint32_t)a.count;
    for (uint32_t which = blockIdx.x; which < count; which += gridDim.x) {
        const int cell = a.list ? a.list[which] : (int)which;
        const int lo = a.cell_start[cell];
        const int n = a.cell_start[cell + 1] - lo;
        if (n > RELAX_LDS_CAP) continue;
        if (n < 2) {
            if (threadIdx.x == 0) a.r_out[cell] = 0.0;
            __syncthreads();
            continue;
        }
        const R *vx = (const R *)a.v + lo;
        const R *vy = (const R *)a.v + a.n + lo;
        const R *vz = (const R *)a.v + 2 * a.n + lo;
        double s5[5] = {0, 0, 0, 0, 0};
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const double x = vx[i], y = vy[i], z = vz[i];
            s5[1] += x;
            s5[2] += y;
            s5[3] += z;
            s5[4] += x * x + y * y + z * z;
        }
        block_sum<5>(s5, red);
        if (threadIdx.x == 0) {
            const double N = (double)n;
            const double T = (s5[4] / N - (s5[1] * s5[1] + s5[2] * s5[2] + s5[3] * s5[3]) / (N * N)) / 3.0;
            double acc[6] = {0, 0, 0, 0, 0, 0};
            const double *pc = a.part + (size_t)which * a.replicas * 6;
            for (int rep = 0; rep < a.replicas; ++rep)
                for (int c = 0; c < 6; ++c) acc[c] += pc[rep * 6 + c];
            const double K = (double)a.replicas;
            double f2 = 0.0;
            for (int c = 0; c < 3; ++c) f2 += (acc[c] / K) * (acc[c] / K);
            for (int c = 3; c < 6; ++c) f2 += 2.0 * (acc[c] / K) * (acc[c] / K);
            a.r_out[cell] = T > 0.0 ? sqrt(f2) / (N * T) : 0.0;
        }
        __syncthreads();
    }
}

// Cells above RELAX_LDS_CAP members: one workgroup per listed cell: r = || (1/K) sum_replicas sum_pairs
// 1/4 h(s^2) (|u|^2 I - 3 u u^T) ||_F / (N T), pairs from independent
// re-pairings (domain 3, c3 = replica); s^2 = 8 pi n lnL dt dt_scale / |u|^3.
template <typename R>
__global__ __launch_bounds__(1024) void k_relax(RelaxArgs a, HugeScratch hs)
{
    __shared__ double red[6 * 16];
    __shared__ uint32_t wtot[16];
    if (relax_off(a)) return;
    const uint64_t step = a.step_dev ? *a.step_dev : a.step;
    const R *vx = (const R *)a.v;
    const R *vy = vx + a.n;
    const R *vz = vy + a.n;
    const int32_t *mine = a.cls_list + 2 * (int64_t)a.cap;
    for (uint32_t item = blockIdx.x; item < a.cls_count[2]; item += gridDim.x) {
        const int cell = relax_cell(a, (uint32_t)mine[item]);
        const int lo = a.cell_start[cell];
        const int n = a.cell_start[cell + 1] - lo;
        // temperature of the cell
        double s5[5] = {0, 0, 0, 0, 0};
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const double x = vx[lo + i], y = vy[lo + i], z = vz[lo + i];
            s5[1] += x;
            s5[2] += y;
            s5[3] += z;
            s5[4] += x * x + y * y + z * z;
        }
        block_sum<5>(s5, red);
        const double N = (double)n;
        const double T = (s5[4] / N - (s5[1] * s5[1] + s5[2] * s5[2] + s5[3] * s5[3]) / (N * N)) / 3.0;
        const double dens = a.density ? a.density[cell] : 1.0;
        const double dts = a.dt_scale ? a.dt_scale[cell] : 1.0;
        const double C = 8.0 * PI_D * dens * a.lnL * a.dt * dts;
        double acc[6] = {0, 0, 0, 0, 0, 0};   // xx yy zz xy xz yz
        for (int rep = 0; rep < a.replicas; ++rep) {
            for (int i = threadIdx.x; i < n; i += blockDim.x)
                hs.keys[lo + i] = draw4(a.seed, a.pid[lo + i], (uint32_t)step, 3u, (uint32_t)rep).x;
            __syncthreads();
            gsort_positions(hs, a.pid, lo, n, wtot);
            for (int q = threadIdx.x; q < n / 2; q += blockDim.x) {
                const int ia = lo + (int)hs.lst[lo + 2 * q], ib = lo + (int)hs.lst[lo + 2 * q + 1];
                const double ux = (double)vx[ia] - (double)vx[ib];
                const double uy = (double)vy[ia] - (double)vy[ib];
                const double uz = (double)vz[ia] - (double)vz[ib];
                const double uu = ux * ux + uy * uy + uz * uz;
                if (uu == 0.0) continue;
                const double hq = 0.25 * h_angle(C / (uu * sqrt(uu)));
                acc[0] += hq * (uu - 3.0 * ux * ux);
                acc[1] += hq * (uu - 3.0 * uy * uy);
                acc[2] += hq * (uu - 3.0 * uz * uz);
                acc[3] += hq * (-3.0 * ux * uy);
                acc[4] += hq * (-3.0 * ux * uz);
                acc[5] += hq * (-3.0 * uy * uz);
            }
            __syncthreads();
        }
        block_sum<6>(acc, red);
        if (threadIdx.x == 0) {
            const double K = (double)a.replicas;
            double f2 = 0.0;
            for (int c = 0; c < 3; ++c) f2 += (acc[c] / K) * (acc[c] / K);
            for (int c = 3; c < 6; ++c) f2 += 2.0 * (acc[c] / K) * (acc[c] / K);
            a.r_out[cell] = T > 0.0 ? sqrt(f2) / (N * T) : 0.0;
        }
        __syncthreads();
    }
}

// Scores the judged cells: a judged cell the network wanted to skip is a
// false skip when its relaxation reaches the tolerance.  With enough judged
// skips and a false-skip fraction above max_false the gate switches itself off.
__global__ void k_gate_score(DevGate *g, const int32_t *__restrict__ judge_list,
                             const uint8_t *__restrict__ want, const double *__restrict__ r,
                             double tol, double max_false, uint32_t min_judged)
{
    __shared__ unsigned long long s_w, s_f;
    if (threadIdx.x == 0) {
        s_w = 0;
        s_f = 0;
    }
    __syncthreads();
    const uint32_t cnt = g->judge_count;
    for (uint32_t k = threadIdx.x; k < cnt; k += blockDim.x) {
        const int j = judge_list[k];
        if (want[j] & 1u) {
            atomicAdd(&s_w, 1ull);
            if (r[j] >= tol) atomicAdd(&s_f, 1ull);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        g->judged += cnt;
        g->judged_want += s_w;
        g->false_skip += s_f;
        if (g->judged_want >= min_judged && (double)g->false_skip > max_false * (double)g->judged_want)
            g->disabled = 1;
        g->steps += 1;
    }
}

__global__ void k_gate_end(DevGate *g)
{
    if (threadIdx.x == 0 && g->mom_now) g->have_moments = 1;
}

// The moment sums are refreshed on the first gated step and then every
// mom_every steps; in between the network reads the last refresh.
__global__ void k_mom_select(DevGate *g, const uint64_t *step_dev, uint64_t step, int every)
{
    if (threadIdx.x == 0) {
        const uint64_t s = step_dev ? *step_dev : step;
        g->mom_now = (!g->have_moments || every <= 1 || s % (uint64_t)every == 0) ? 1 : 0;
    }
}

// ------------------------------------------------------------ training
// One block: a tile of TS samples; forward, loss and backward with the
// activations in LDS, partial gradients written per tile and summed in a
// fixed order by k_reduce_grads (bitwise reproducible).
constexpr int TS = 64;

__global__ __launch_bounds__(256) void k_mlp_grad_tile(const float *__restrict__ params,
                                                      const float *__restrict__ x,
                                                      const float *__restrict__ y, int32_t B,
                                                      int bf16, float *__restrict__ partial,
                                                      float *__restrict__ loss_partial)
{
    __shared__ float P[NPARAM];
    __shared__ float X[TS * 8];
    __shared__ float Z1[TS * 64], A1[TS * 64], Z2[TS * 64], A2[TS * 64];
    __shared__ float D3[TS];
    __shared__ float Ls[TS];
    const bool b16 = bf16 != 0;
    load_params(P, params, b16);
    const int s0 = blockIdx.x * TS;
    const int ns = min(TS, B - s0);
    for (int e = threadIdx.x; e < TS * 8; e += blockDim.x) {
        const int s = e / 8;
        const float v = s < ns ? x[(int64_t)(s0 + s) * 8 + (e % 8)] : 0.0f;
        X[e] = b16 ? bf16r(v) : v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < TS * 64; e += blockDim.x) {
        const int s = e / 64, j = e % 64;
        float z = P[OFF_B1 + j];
        for (int i = 0; i < 8; ++i) z += X[s * 8 + i] * P[OFF_W1 + i * 64 + j];
        Z1[e] = z;
        const float r = z > 0.0f ? z : 0.0f;
        A1[e] = b16 ? bf16r(r) : r;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < TS * 64; e += blockDim.x) {
        const int s = e / 64, j = e % 64;
        float z = P[OFF_B2 + j];
        for (int i = 0; i < 64; ++i) z += A1[s * 64 + i] * P[OFF_W2 + i * 64 + j];
        Z2[e] = z;
        const float r = z > 0.0f ? z : 0.0f;
        A2[e] = b16 ? bf16r(r) : r;
    }
    __syncthreads();
    if (threadIdx.x < TS) {
        const int s = threadIdx.x;
        float d = 0.0f, l = 0.0f;
        if (s < ns) {
            float z = P[OFF_B3];
            for (int j = 0; j < 64; ++j) z += A2[s * 64 + j] * P[OFF_W3 + j];
            const float p = 1.0f / (1.0f + __expf(-z));
            const float t = y[s0 + s];
            l = fmaxf(z, 0.0f) - z * t + log1pf(__expf(-fabsf(z)));
            d = (p - t) / (float)B;
        }
        D3[s] = b16 ? bf16r(d) : d;
        Ls[s] = l;
    }
    __syncthreads();
    float *G = partial + (int64_t)blockIdx.x * NPARAM;
    // layer 3
    if (threadIdx.x < 64) {
        const int j = threadIdx.x;
        float g = 0.0f;
        for (int s = 0; s < TS; ++s) g += A2[s * 64 + j] * D3[s];
        G[OFF_W3 + j] = g;
    }
    if (threadIdx.x == 64) {
        float g = 0.0f, l = 0.0f;
        for (int s = 0; s < TS; ++s) {
            g += D3[s];
            l += Ls[s];
        }
        G[OFF_B3] = g;
        loss_partial[blockIdx.x] = l;
    }
    __syncthreads();
    // delta of layer 2 (overwrites Z2)
    for (int e = threadIdx.x; e < TS * 64; e += blockDim.x) {
        const int s = e / 64, j = e % 64;
        const float d = Z2[e] > 0.0f ? P[OFF_W3 + j] * D3[s] : 0.0f;
        Z2[e] = b16 ? bf16r(d) : d;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
        const int i = e / 64, j = e % 64;
        float g = 0.0f;
        for (int s = 0; s < TS; ++s) g += A1[s * 64 + i] * Z2[s * 64 + j];
        G[OFF_W2 + e] = g;
    }
    if (threadIdx.x < 64) {
        float g = 0.0f;
        for (int s = 0; s < TS; ++s) g += Z2[s * 64 + threadIdx.x];
        G[OFF_B2 + threadIdx.x] = g;
    }
    // delta of layer 1 (overwrites Z1)
    for (int e = threadIdx.x; e < TS * 64; e += blockDim.x) {
        const int s = e / 64, i = e % 64;
        float d = 0.0f;
        if (Z1[e] > 0.0f) {
            for (int j = 0; j < 64; ++j) d += P[OFF_W2 + i * 64 + j] * Z2[s * 64 + j];
        }
        Z1[e] = b16 ? bf16r(d) : d;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 8 * 64; e += blockDim.x) {
        const int i = e / 64, j = e % 64;
        float g = 0.0f;
        for (int s = 0; s < TS; ++s) g += X[s * 8 + i] * Z1[s * 64 + j];
        G[OFF_W1 + e] = g;
    }
    if (threadIdx.x < 64) {
        float g = 0.0f;
        for (int s = 0; s < TS; ++s) g += Z1[s * 64 + threadIdx.x];
        G[OFF_B1 + threadIdx.x] = g;
    }
}

__global__ void k_reduce_grads(const float *__restrict__ partial, const float *__restrict__ loss_partial,
                               int tiles, int32_t B, float *__restrict__ grad, float *__restrict__ loss)
{
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < NPARAM; p += gridDim.x * blockDim.x) {
        float g = 0.0f;
        for (int t = 0; t < tiles; ++t) g += partial[(int64_t)t * NPARAM + p];
        grad[p] = g;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && loss) {
        float l = 0.0f;
        for (int t = 0; t < tiles; ++t) l += loss_partial[t];
        *loss = l / (float)B;
    }
}

// Adam (Kingma & Ba) with bias correction, step t >= 1.
__global__ void k_adam(float *__restrict__ params, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ grad, int32_t t, float lr, float b1, float b2, float eps)
{
    const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < NPARAM; p += gridDim.x * blockDim.x) {
        const float g = grad[p];
        const float mm = b1 * m[p] + (1.0f - b1) * g;
        const float vv = b2 * v[p] + (1.0f - b2) * g * g;
        m[p] = mm;
        v[p] = vv;
        params[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    }
}

}  // namespace

int launch_features(const double *moments, int32_t M, float *feat, uint8_t *valid, hipStream_t st)
{
    const int g = (M + 255) / 256 < 4096 ? (M + 255) / 256 : 4096;
    hipLaunchKernelGGL(k_features, dim3(g > 0 ? g : 1), dim3(256), 0, st, moments, M, feat, valid);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

namespace {
// skip = p > thr and fewer than kmax deferred steps; the count follows.
__global__ void k_gate_infer_decide(const float *__restrict__ prob, int32_t M, float thr, int32_t kmax,
                                    uint8_t *__restrict__ skip, int32_t *__restrict__ k_acc)
{
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < M; j += gridDim.x * blockDim.x) {
        const bool s = prob[j] > thr && k_acc[j] < kmax;
        skip[j] = s;
        k_acc[j] = s ? k_acc[j] + 1 : 0;
    }
}
}  // namespace

int launch_gate_infer_decide(const float *prob, int32_t M, float thr, int32_t kmax, uint8_t *skip,
                             int32_t *k_acc, hipStream_t st)
{
    if (M <= 0) return PIC_OK;
    const int g = (M + 255) / 256 < 4096 ? (M + 255) / 256 : 4096;
    hipLaunchKernelGGL(k_gate_infer_decide, dim3(g), dim3(256), 0, st, prob, M, thr, kmax, skip, k_acc);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

int launch_mlp_forward(const float *params, const float *x, int32_t B, int bf16, float *prob,
                       hipStream_t st)
{
    if (B <= 0) return PIC_OK;
    if (bf16) {
        const int tiles = (B + 31) / 32;
        const int g = (tiles + 3) / 4 < 1024 ? (tiles + 3) / 4 : 1024;
        hipLaunchKernelGGL(k_mlp_forward_mfma, dim3(g), dim3(256), 0, st, params, x, B, prob);
    } else {
        const int g = (B + 255) / 256 < 1024 ? (B + 255) / 256 : 1024;
        hipLaunchKernelGGL(k_mlp_forward, dim3(g), dim3(256), 0, st, params, x, B, bf16, prob);
    }
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

size_t mlp_grad_scratch_floats(int32_t B)
{
    const int tiles = (B + TS - 1) / TS;
    return (size_t)tiles * NPARAM + tiles + NPARAM + 64;
}

int launch_mlp_grad(const float *params, const float *x, const float *y, int32_t B, int bf16,
                    float *scratch, float *grad, float *loss, hipStream_t st)
{
    const int tiles = (B + TS - 1) / TS;
    float *partial = scratch;
    float *lp = scratch + (size_t)tiles * NPARAM;
    hipLaunchKernelGGL(k_mlp_grad_tile, dim3(tiles), dim3(256), 0, st, params, x, y, B, bf16, partial, lp);
    hipLaunchKernelGGL(k_reduce_grads, dim3((NPARAM + 255) / 256), dim3(256), 0, st, partial, lp, tiles,
                       B, grad, loss);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

int launch_adam(float *params, float *m, float *v, const float *grad, int32_t t, float lr,
                hipStream_t st)
{
    hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, st, params, m, v, grad, t, lr,
                       0.9f, 0.999f, 1e-8f);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

int launch_analytic_relax(const double *moments, int32_t M, double dt, double lnL, const double *density,
                          int replicas, double *r, hipStream_t st)
{
    const int g = (M + 255) / 256 < 2048 ? (M + 255) / 256 : 2048;
    hipLaunchKernelGGL(k_analytic_relax, dim3(g > 0 ? g : 1), dim3(256), 0, st, moments, M, dt, lnL,
                       density, replicas, r);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

int launch_gate(const GateArgs &a, hipStream_t st)
{
    if (a.analytic) {
        const int g = (a.M + 255) / 256 < 2048 ? (a.M + 255) / 256 : 2048;
        hipLaunchKernelGGL(k_gate_analytic, dim3(g > 0 ? g : 1), dim3(256), 0, st, a);
    } else if (a.bf16) {
        const int tiles = (a.M + 31) / 32;
        const int g = (tiles + 3) / 4 < 1024 ? (tiles + 3) / 4 : 1024;
        hipLaunchKernelGGL(k_gate_mfma, dim3(g > 0 ? g : 1), dim3(256), 0, st, a);
    } else {
        const int g = (a.M + 255) / 256 < 2048 ? (a.M + 255) / 256 : 2048;
        hipLaunchKernelGGL(k_gate, dim3(g > 0 ? g : 1), dim3(256), 0, st, a);
    }
    hipLaunchKernelGGL(k_gate_list, dim3(1), dim3(1024), 0, st, a.g, a.want, a.skip, a.M, a.judge_list);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

int launch_gate_score(DevGate *g, const int32_t *judge_list, const uint8_t *want, const double *r,
                      double tol, double max_false, uint32_t min_judged, hipStream_t st)
{
    hipLaunchKernelGGL(k_gate_score, dim3(1), dim3(256), 0, st, g, judge_list, want, r, tol, max_false,
                       min_judged);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

int launch_mom_select(DevGate *g, const uint64_t *step_dev, uint64_t step, int every, hipStream_t st)
{
    hipLaunchKernelGGL(k_mom_select, dim3(1), dim3(64), 0, st, g, step_dev, step, every);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

int launch_gate_end(DevGate *g, hipStream_t st)
{
    hipLaunchKernelGGL(k_gate_end, dim3(1), dim3(64), 0, st, g);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

size_t relax_part_bytes(int64_t count, int replicas)
{
    return (size_t)count * (size_t)replicas * 6 * sizeof(double) + 3 * (size_t)count * 4 + 16 + 256;
}

template <typename R, int T, int K>
static int launch_relax_lds(const RelaxArgs &a, int cls, int blocks, hipStream_t st)
{
    const size_t lds = sort_bytes(T * K);
    auto kern = k_relax_lds<R, T, K>;
    static bool attr_done = false;
    if (!attr_done) {
        HIP_OK(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds));
        attr_done = true;
    }
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(T), lds, st, a, cls);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

template <typename R>
static int launch_relax_t(const RelaxArgs &a0, int num_cu, hipStream_t st)
{
    int rc;
    // class lists and counts follow the per-replica sums in the scratch
    RelaxArgs a = a0;
    a.cls_list = (int32_t *)(a.part + (size_t)a.cap * a.replicas * 6);
    a.cls_count = (uint32_t *)(a.cls_list + 3 * (size_t)a.cap);
    hipLaunchKernelGGL(k_relax_classify, dim3(1), dim3(RELAX_CLASSIFY_T), 0, st, a);
    if ((rc = launch_relax_lds<R, RELAX_T0, RELAX_K0>(a, 0, num_cu * 6, st))) return rc;
    if ((rc = launch_relax_lds<R, RELAX_T1, RELAX_K1>(a, 1, num_cu, st))) return rc;
    hipLaunchKernelGGL(k_relax<R>, dim3(num_cu), dim3(1024), 0, st, a, huge_scratch());
    hipLaunchKernelGGL(k_relax_finish<R>, dim3(num_cu * 4), dim3(256), 0, st, a);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

int launch_relax(int dtype, const RelaxArgs &a, int num_cu, hipStream_t st)
{
    return dtype == PIC_F32 ? launch_relax_t<float>(a, num_cu, st) : launch_relax_t<double>(a, num_cu, st);
}

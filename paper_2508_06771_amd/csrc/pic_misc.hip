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

// ------------------------------------------------------------ recombination
// Recombination C5 on cell-sorted storage, one workgroup per cell.  The
// paper pops catalytes from per-cell lists with atomics; here the matching
// is fixed: the k-th live primary of the cell in storage order takes the
// live catalyte of rank (o_j + k) mod C_j, o_j = floor(word0 C_j / 2^32) of
// a domain-9 draw on the cell index, for k < min(P_j, C_j).  Each wave walks
// a quarter of the cell with a running count (ballots, no barriers), keeping
// each 64-member chunk's primary and catalyte ballots in LDS; the quarters'
// counts give each wave its starting ranks, and the later passes rank from
// the kept ballots instead of reading the cell again.  Primaries of ranks
// [k0, k0 + RC_CAP) are parked in LDS, then the catalytes matched to them
// are updated: energy |v_c|^2/2 + |v_p|^2/2 + eps, isotropic direction from
// words 1, 2 of a domain-8 draw on the catalyte's pid; the matched
// primaries' weights become 0 at the end.
constexpr int RC_T = 256;
constexpr int RC_W = RC_T / PIC_WAVE;
constexpr int RC_CAP = 2048;
constexpr int RC_U = 8;   // 64-member chunks whose loads are in flight together

// Walks members [qs, qe) in 64-member chunks, calling f(l, alive, primary)
// with the whole wave for each chunk in order until f returns false (f's
// result must be the same on every lane).  The loads of RC_U chunks are
// issued together, past-the-end lanes reloading member qe - 1 (masked).
template <typename R, typename F>
__device__ __forceinline__ void rc_walk(const R *__restrict__ w, const uint8_t *__restrict__ primary, int64_t qs,
                                        int64_t qe, F &&f)
{
    const int lane = threadIdx.x & (PIC_WAVE - 1);
    for (int64_t i0 = qs; i0 < qe; i0 += RC_U * PIC_WAVE) {
        R wv[RC_U];
        uint8_t pv[RC_U];
#pragma unroll
        for (int u = 0; u < RC_U; ++u) {
            int64_t l = i0 + u * PIC_WAVE + lane;
            l = l < qe ? l : qe - 1;
            wv[u] = w[l];
            pv[u] = primary[l];
        }
#pragma unroll
        for (int u = 0; u < RC_U; ++u) {
            const int64_t l = i0 + u * PIC_WAVE + lane;
            const bool alive = l < qe && wv[u] > (R)0;
            if (!f(l, alive, alive && pv[u] != 0)) return;
        }
    }
}

constexpr int RC_MAXC = 128;   // 64-member chunks per wave whose ballots stay in LDS (8 KB)

template <typename R>
__global__ __launch_bounds__(RC_T) void k_recombine(RecombArgs a)
{
#pragma clang fp contract(off)
    __shared__ uint32_t s_prim[RC_CAP];
    __shared__ uint32_t s_cnt[2 * RC_W];
    __shared__ uint64_t s_pm[RC_W][RC_MAXC], s_cm[RC_W][RC_MAXC];   // primary / catalyte ballots
    R *v = (R *)a.v;
    R *w = (R *)a.w;
    const int64_t n = a.n;
    const int lane = threadIdx.x & (PIC_WAVE - 1), wid = threadIdx.x / PIC_WAVE;
    const uint64_t below = (1ull << lane) - 1ull;
    for (int32_t j = blockIdx.x; j < a.M; j += gridDim.x) {
        const int64_t s = a.cs[j], e = a.cs[j + 1];
        const int64_t q = (e - s + RC_W - 1) / RC_W;
        const int64_t qs = s + wid * q, qe = qs + q < e ? qs + q : e;
        // count pass: the only full read of the cell; the chunks' ballots are
        // kept (the first RC_MAXC chunks of each wave) for the later passes
        uint32_t P = 0, C = 0, k = 0;
        rc_walk(w, a.primary, qs, qe, [&](int64_t, bool alive, bool pr) {
            const uint64_t pm = __ballot(pr), cm = __ballot(alive && !pr);
            if (k < RC_MAXC && lane == 0) {
                s_pm[wid][k] = pm;
                s_cm[wid][k] = cm;
            }
            ++k;
            P += (uint32_t)__popcll(pm);
            C += (uint32_t)__popcll(cm);
            return true;
        });
        const uint32_t nk = k;
        // chunk kk's ballots: from LDS, or re-read past the kept ones (the
        // weights are only written by the last pass, which ranks by them first)
        auto masks = [&](uint32_t kk, uint64_t &pm, uint64_t &cm) {
            if (kk < RC_MAXC) {
                pm = s_pm[wid][kk];
                cm = s_cm[wid][kk];
            } else {
                const int64_t l = qs + (int64_t)kk * PIC_WAVE + lane;
                const bool alive = l < qe && w[l] > (R)0;
                const bool pr = alive && a.primary[l] != 0;
                pm = __ballot(pr);
                cm = __ballot(alive && !pr);
            }
        };
        if (lane == 0) {
            s_cnt[wid] = P;
            s_cnt[RC_W + wid] = C;
        }
        __syncthreads();
        uint32_t Pt = 0, Ct = 0, Pb = 0, Cb = 0;
#pragma unroll
        for (int x = 0; x < RC_W; ++x) {
            Pt += s_cnt[x];
            Ct += s_cnt[RC_W + x];
            if (x < wid) {
                Pb += s_cnt[x];
                Cb += s_cnt[RC_W + x];
            }
        }
        const uint32_t m = Pt < Ct ? Pt : Ct;
        if (threadIdx.x == 0 && a.events) a.events[j] = (int32_t)m;
        if (m > 0) {
            const uint32_t o = (uint32_t)(((uint64_t)draw4(a.seed, (uint32_t)j, a.step, 9u, 0u).x * Ct) >> 32);
            for (uint32_t k0 = 0; k0 < m; k0 += RC_CAP) {
                const uint32_t k1 = m < k0 + RC_CAP ? m : k0 + RC_CAP;
                uint32_t r0 = Pb;   // rank of this wave's next primary
                for (uint32_t kk = 0; kk < nk && r0 < k1; ++kk) {
                    uint64_t pm, cm;
                    masks(kk, pm, cm);
                    const uint32_t r = r0 + (uint32_t)__popcll(pm & below);
                    if ((pm >> lane) & 1ull && r >= k0 && r < k1)
                        s_prim[r - k0] = (uint32_t)(qs + (int64_t)kk * PIC_WAVE + lane);
                    r0 += (uint32_t)__popcll(pm);
                }
                __syncthreads();
                uint32_t c0 = Cb;   // rank of this wave's next catalyte
                for (uint32_t kk = 0; kk < nk; ++kk) {
                    uint64_t pm, cm;
                    masks(kk, pm, cm);
                    const uint32_t r = c0 + (uint32_t)__popcll(cm & below);
                    c0 += (uint32_t)__popcll(cm);
                    if (!((cm >> lane) & 1ull)) continue;
                    const uint32_t kc = (uint32_t)(((uint64_t)r + Ct - o) % Ct);
                    if (kc < k0 || kc >= k1) continue;
                    const int64_t l = qs + (int64_t)kk * PIC_WAVE + lane;
                    const int64_t p = s_prim[kc - k0];
                    const double px = v[p], py = v[n + p], pz = v[2 * n + p];
                    const double cx = v[l], cy = v[n + l], cz = v[2 * n + l];
                    const double ep = 0.5 * (px * px + py * py + pz * pz);
                    const double ec = 0.5 * (cx * cx + cy * cy + cz * cz);
                    const double sp = sqrt(2.0 * (ec + ep + a.eps));
                    const W4 dw = draw4(a.seed, a.pid[l], a.step, 8u, 0u);
                    double sx, sy, sz;
                    dsmc_dir(dw.y, dw.z, sx, sy, sz);
                    v[l] = (R)(sp * sx);
                    v[n + l] = (R)(sp * sy);
                    v[2 * n + l] = (R)(sp * sz);
                }
                __syncthreads();   // s_prim is refilled by the next round
            }
            // the matched primaries are the first m: their weights go to 0
            // only now, so every round above ranked the same live primaries
            uint32_t r0 = Pb;
            for (uint32_t kk = 0; kk < nk && r0 < m; ++kk) {
                uint64_t pm, cm;
                masks(kk, pm, cm);
                const uint32_t r = r0 + (uint32_t)__popcll(pm & below);
                r0 += (uint32_t)__popcll(pm);
                if ((pm >> lane) & 1ull && r < m) w[qs + (int64_t)kk * PIC_WAVE + lane] = (R)0;
            }
        }
        __syncthreads();   // s_cnt and the masks are rewritten for the next cell
    }
}

// ------------------------------------------------------------ Nanbu
// ------------------------------------------------------------ exact count
// The k smallest candidate words.  The words are uniform, so the k-th lies
// within a few binomial standard deviations of k 2^32 / n: one pass draws
// every word and sorts it into "below the window" (selected; slot appended to
// the workgroup's list), "in the window" (word, pid and slot appended to the
// workgroup's short list) or "above" (not selected).  One workgroup then
// finds the exact threshold among the window words by radix selection; only
// when the window missed (the count below it exceeds k, the count up to its
// top falls short of k, or a workgroup's list overflowed) does it select over
// every particle, re-drawing the words.  Nothing is written to v before the
// decision, so both outcomes are exact.  The lists are per workgroup, with
// LDS counters, because a single global counter serialises in L2.
struct ExactState {
    uint32_t n_x;        // tie winners (window mode)
    uint32_t n_win;      // compacted window words
    uint32_t fallback;   // the window missed: select over all particles
    uint32_t t;          // threshold word
    uint32_t krem;       // words equal to t still to select (fallback)
    uint32_t n_ties;     // words equal to t (fallback)
    uint32_t pad[2];
};

struct ExactBufs {
    uint32_t *lo_slot;    // G x cap_lo slots below the window
    uint32_t *win_key;    // G x cap_win window words
    uint64_t *win_ps;     // G x cap_win (pid << 32) | slot
    uint32_t *cnt_lo;     // G counts (may exceed cap_lo: overflow)
    uint32_t *cnt_win;    // G counts
    uint32_t *ckey;       // compacted window words
    uint64_t *cps;        // compacted (pid << 32) | slot
    uint32_t *x_slot;     // tie winners (k slots)
    uint64_t *ties;       // n entries of (pid << 32) | slot
    ExactState *st;
    uint64_t lo, hi;      // window [lo, hi) of words, 0 <= lo <= hi <= 2^32
    int64_t chunk;        // particles per workgroup
    uint32_t k, cap_lo, cap_win, G;
};

constexpr int SEL_BINS = 2048;
constexpr int SEL_T = 1024;
constexpr int SEL_LDS = 12288;   // window words kept in LDS (48 KB)
constexpr int EXACT_G = 2048;    // workgroups of the classify and scatter passes, at most

// Index of this lane's entry when the lanes with p set append to a list
// through one LDS counter (one atomic per wave).
__device__ __forceinline__ uint32_t wave_append(bool p, uint32_t *ctr)
{
    const uint64_t m = __ballot(p);
    if (!m) return 0u;
    const int lane = threadIdx.x & (PIC_WAVE - 1);
    const int leader = __ffsll((unsigned long long)m) - 1;
    uint32_t base = 0u;
    if (lane == leader) base = atomicAdd(ctr, (uint32_t)__popcll(m));
    base = __shfl(base, leader);
    return base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
}

__global__ __launch_bounds__(256) void k_exact_classify(const uint32_t *__restrict__ pid, int64_t n,
                                                        uint64_t seed, uint32_t step, ExactBufs b,
                                                        uint8_t *__restrict__ sel_out)
{
    __shared__ uint32_t s_lo, s_win;
    if (threadIdx.x == 0) {
        s_lo = 0u;
        s_win = 0u;
    }
    __syncthreads();
    const int64_t start = blockIdx.x * b.chunk;
    const int64_t end = start + b.chunk < n ? start + b.chunk : n;
    uint32_t *lo_out = b.lo_slot + (size_t)blockIdx.x * b.cap_lo;
    uint32_t *wk = b.win_key + (size_t)blockIdx.x * b.cap_win;
    uint64_t *wp = b.win_ps + (size_t)blockIdx.x * b.cap_win;
    for (int64_t l = start + threadIdx.x; l < end; l += blockDim.x) {
        const uint32_t p = pid[l];
        const uint32_t key = draw4(seed, p, step, 0u, 0u).y;
        const bool below = (uint64_t)key < b.lo;
        const bool inwin = !below && (uint64_t)key < b.hi;
        const uint32_t i = wave_append(below, &s_lo);
        if (below && i < b.cap_lo) lo_out[i] = (uint32_t)l;
        const uint32_t j = wave_append(inwin, &s_win);
        if (inwin && j < b.cap_win) {
            wk[j] = key;
            wp[j] = ((uint64_t)p << 32) | (uint64_t)l;
        }
        if (sel_out) sel_out[l] = below;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        b.cnt_lo[blockIdx.x] = s_lo;
        b.cnt_win[blockIdx.x] = s_win;
    }
}

// One workgroup of SEL_T threads.  Window mode: the r = k - n_lo smallest
// window words by (word, pid, slot) go to x_slot.  Fallback: the threshold
// word t over all particles and, of the words equal to t, how many to take;
// the scatter pass then decides every particle.
__global__ __launch_bounds__(SEL_T) void k_exact_select(const uint32_t *__restrict__ pid, int64_t n,
                                                        uint64_t seed, uint32_t step, ExactBufs b)
{
    __shared__ uint32_t h[SEL_BINS];        // list prefixes, then the histogram
    __shared__ uint32_t s_key[SEL_LDS];
    __shared__ uint32_t wtot[SEL_T / PIC_WAVE];
    __shared__ uint32_t s_digit, s_before, s_nt, s_nx, s_over, s_nlo, s_nwin;
    ExactState *st = b.st;
    // totals over the workgroups' lists (two lists a thread)
    const uint32_t b0 = 2 * threadIdx.x, b1 = b0 + 1;
    const uint32_t l0 = b0 < b.G ? b.cnt_lo[b0] : 0u, l1 = b1 < b.G ? b.cnt_lo[b1] : 0u;
    const uint32_t w0 = b0 < b.G ? b.cnt_win[b0] : 0u, w1 = b1 < b.G ? b.cnt_win[b1] : 0u;
    if (threadIdx.x == 0) s_over = 0u;
    __syncthreads();
    if (l0 > b.cap_lo || l1 > b.cap_lo || w0 > b.cap_win || w1 > b.cap_win) s_over = 1u;
    const uint32_t exl = block_excl(l0 + l1, wtot);
    if (threadIdx.x == SEL_T - 1) s_nlo = exl + l0 + l1;
    const uint32_t exw = block_excl(w0 + w1, wtot);
    if (threadIdx.x == SEL_T - 1) s_nwin = exw + w0 + w1;
    if (b0 < SEL_BINS) h[b0] = exw;
    if (b1 < SEL_BINS) h[b1] = exw + w0;
    __syncthreads();
    const uint32_t n_lo = s_nlo, n_win = s_nwin;
    const bool fb = s_over || !(n_lo <= b.k && (uint64_t)n_lo + n_win >= b.k);
    const uint32_t r = fb ? b.k : b.k - n_lo;
    if (r == 0) {   // nothing beyond the lists below the window
        if (threadIdx.x == 0) {
            st->n_x = 0u;
            st->n_win = 0u;
            st->fallback = 0u;
        }
        return;
    }
    const bool in_lds = n_win <= (uint32_t)SEL_LDS;
    if (!fb) {
        // compact the window lists (the last list whose prefix is <= i holds
        // entry i), four entries a thread in flight
        for (uint32_t i0 = 0; i0 < n_win; i0 += 4 * SEL_T) {
            uint32_t kk[4];
            uint64_t pp[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t i = i0 + u * SEL_T + threadIdx.x;
                if (i < n_win) {
                    uint32_t lo = 0, hi = b.G;   // h[lo] <= i < h[hi]
                    while (hi - lo > 1) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (h[mid] <= i) lo = mid;
                        else hi = mid;
                    }
                    const size_t src = (size_t)lo * b.cap_win + (i - h[lo]);
                    kk[u] = b.win_key[src];
                    pp[u] = b.win_ps[src];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t i = i0 + u * SEL_T + threadIdx.x;
                if (i < n_win) {
                    if (in_lds) s_key[i] = kk[u];
                    b.ckey[i] = kk[u];
                    b.cps[i] = pp[u];
                }
            }
        }
        __syncthreads();
    }
    const int64_t count = fb ? n : (int64_t)n_win;
    auto key_at = [&](int64_t i) -> uint32_t {
        return fb ? draw4(seed, pid[i], step, 0u, 0u).y : in_lds ? s_key[i] : b.ckey[i];
    };
    // digits of the word minus the window's base, over the bits its span
    // needs (a narrow window's words share their top bits, and a histogram
    // of those would pile into one LDS bin); 11-bit digits from the top
    const uint32_t base = fb ? 0u : (uint32_t)b.lo;
    const uint64_t span = fb ? (uint64_t)1 << 32 : b.hi - b.lo;
    const int nbits = span <= 1 ? 1 : 64 - __clzll((long long)(span - 1));
    const int npass = (nbits + 10) / 11;
    uint32_t prefix = 0u, krem = r;
    for (int pass = 0; pass < npass; ++pass) {
        const int above = nbits - 11 * pass;
        const int shift = above > 11 ? above - 11 : 0;
        const int bits = above - shift;
        for (int i = threadIdx.x; i < SEL_BINS; i += SEL_T) h[i] = 0u;
        __syncthreads();
        for (int64_t i = threadIdx.x; i < count; i += SEL_T) {
            const uint32_t key = key_at(i) - base;
            if (pass == 0 || (key >> above) == prefix)
                atomicAdd(&h[(key >> shift) & ((1u << bits) - 1u)], 1u);
        }
        __syncthreads();
        // the first bin whose inclusive count reaches krem (two bins a thread)
        const uint32_t nb = 1u << bits;
        const uint32_t c0 = b0 < nb ? h[b0] : 0u, c1 = b1 < nb ? h[b1] : 0u;
        const uint32_t ex = block_excl(c0 + c1, wtot);
        if (b0 < nb && ex < krem && ex + c0 >= krem) {
            s_digit = b0;
            s_before = ex;
        }
        if (b1 < nb && ex + c0 < krem && ex + c0 + c1 >= krem) {
            s_digit = b1;
            s_before = ex + c0;
        }
        __syncthreads();
        prefix = (prefix << bits) | s_digit;
        krem -= s_before;
        __syncthreads();   // s_digit, s_before and h are rewritten by the next pass
    }
    const uint32_t t = prefix + base;
    if (threadIdx.x == 0) {
        s_nt = 0u;
        s_nx = 0u;
    }
    __syncthreads();
    for (int64_t i0 = 0; i0 < count; i0 += SEL_T) {   // uniform trip count: whole waves append
        const int64_t i = i0 + threadIdx.x;
        const bool tie = i < count && key_at(i) == t;
        const uint32_t qt = wave_append(tie, &s_nt);
        if (tie) b.ties[qt] = fb ? (((uint64_t)pid[i] << 32) | (uint64_t)i) : b.cps[i];
    }
    __syncthreads();
    const uint32_t m = s_nt;
    if (!fb) {
        // of the words equal to t, the krem first by (pid, slot)
        for (uint32_t i = threadIdx.x; i < m; i += SEL_T) {
            const uint64_t e = b.ties[i];
            uint32_t rank = 0u;
            for (uint32_t j = 0; j < m; ++j) rank += b.ties[j] < e ? 1u : 0u;
            if (rank < krem) b.x_slot[atomicAdd(&s_nx, 1u)] = (uint32_t)e;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        st->t = t;
        st->krem = krem;
        st->n_ties = m;
        st->n_x = fb ? 0u : s_nx;
        st->n_win = fb ? 0u : n_win;
        st->fallback = fb ? 1u : 0u;
    }
}

template <typename R>
__device__ __forceinline__ void exact_scatter_one(R *__restrict__ v, int64_t n, int64_t l, uint32_t p,
                                                  double mass_ratio, uint64_t seed, uint32_t step)
{
    R x = v[l], y = v[n + l], z = v[2 * n + l];
    scatter_dir(x, y, z, draw4(seed, p, step, 1u, 0u), mass_ratio);
    v[l] = x;
    v[n + l] = y;
    v[2 * n + l] = z;
}

// Window mode: workgroup g scatters its own list below the window, and all
// workgroups share the window words below t and the tie winners.  Fallback:
// every particle, its word re-drawn; equal words ranked by (pid, slot)
// against the collected ties.
template <typename R>
__global__ __launch_bounds__(256) void k_exact_scatter(R *__restrict__ v, const uint32_t *__restrict__ pid,
                                                       int64_t n, ExactBufs b, double mass_ratio, uint64_t seed,
                                                       uint32_t step, uint8_t *__restrict__ sel_out)
{
    const ExactState *st = b.st;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t g0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (!st->fallback) {
        const uint32_t c = b.cnt_lo[blockIdx.x];   // <= cap_lo outside the fallback
        const uint32_t *lo_in = b.lo_slot + (size_t)blockIdx.x * b.cap_lo;
        for (uint32_t i = threadIdx.x; i < c; i += blockDim.x) {
            const int64_t l = lo_in[i];
            exact_scatter_one(v, n, l, pid[l], mass_ratio, seed, step);
        }
        const uint32_t t = st->t;
        const int64_t n_win = st->n_win;
        for (int64_t i = g0; i < n_win; i += stride) {
            if (b.ckey[i] >= t) continue;
            const int64_t l = (uint32_t)b.cps[i];
            if (sel_out) sel_out[l] = 1;
            exact_scatter_one(v, n, l, (uint32_t)(b.cps[i] >> 32), mass_ratio, seed, step);
        }
        const int64_t n_x = st->n_x;
        for (int64_t i = g0; i < n_x; i += stride) {
            const int64_t l = b.x_slot[i];
            if (sel_out) sel_out[l] = 1;
            exact_scatter_one(v, n, l, pid[l], mass_ratio, seed, step);
        }
        return;
    }
    const uint32_t t = st->t, krem = st->krem, m = st->n_ties;
    for (int64_t l = g0; l < n; l += stride) {
        const uint32_t p = pid[l];
        const uint32_t key = draw4(seed, p, step, 0u, 0u).y;
        bool sel = key < t;
        if (key == t) {
            const uint64_t e = ((uint64_t)p << 32) | (uint64_t)l;
            uint32_t rank = 0u;
            for (uint32_t j = 0; j < m; ++j) rank += b.ties[j] < e ? 1u : 0u;
            sel = rank < krem;
        }
        if (sel_out) sel_out[l] = sel;
        if (sel) exact_scatter_one(v, n, l, p, mass_ratio, seed, step);
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

namespace {
struct ExactPlan {
    uint64_t lo, hi;
    int64_t chunk;
    uint32_t k, cap_lo, cap_win, G;
};

// Window of words around the expected k-th: +-8 binomial standard deviations
// of the count, plus 16; per-workgroup list capacities 10 standard
// deviations above their expected fill, plus 32.
ExactPlan exact_plan(int64_t n, int64_t k)
{
    ExactPlan p;
    p.k = (uint32_t)(k < 0 ? 0 : (k > n ? n : k));
    const double nn = (double)n, kk = (double)p.k;
    const double sd = sqrt(kk * (1.0 - kk / nn));
    const double a = (kk - 8.0 * sd - 16.0) / nn, b = (kk + 8.0 * sd + 16.0) / nn;
    const double two32 = 4294967296.0;
    p.lo = a <= 0.0 ? 0 : a >= 1.0 ? (uint64_t)1 << 32 : (uint64_t)floor(a * two32);
    p.hi = b >= 1.0 ? (uint64_t)1 << 32 : (uint64_t)ceil(b * two32);
    if (p.k == 0) p.lo = p.hi = 0;
    int64_t G = (n + 255) / 256;
    if (G > EXACT_G) G = EXACT_G;
    if (G < 1) G = 1;
    p.chunk = (n + G - 1) / G;
    p.G = (uint32_t)((n + p.chunk - 1) / p.chunk);
    auto cap = [&](double frac) {
        const double mu = (double)p.chunk * frac;
        const double c = ceil(mu + 10.0 * sqrt(mu) + 32.0);
        return (uint32_t)(c < (double)p.chunk ? c : (double)p.chunk);
    };
    p.cap_lo = cap((double)p.lo / two32);
    p.cap_win = cap((double)(p.hi - p.lo) / two32);
    return p;
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }
}  // namespace

size_t mcc_exact_ws_bytes(int64_t n, int64_t k)
{
    const ExactPlan p = exact_plan(n, k);
    const size_t win = (size_t)p.G * p.cap_win;
    return round256((size_t)p.G * p.cap_lo * 4) + 2 * round256(win * 4) + 2 * round256(win * 8) +
           2 * round256((size_t)p.G * 4) + round256((size_t)p.k * 4) + round256((size_t)n * 8) +
           round256(sizeof(ExactState));
}

int launch_mcc_exact(int dtype, void *v, const uint32_t *pid, int64_t n, int64_t k, double mass_ratio,
                     uint64_t seed, uint64_t step, uint8_t *selected_out, void *ws, hipStream_t st)
{
    if (n <= 0) return PIC_OK;
    const ExactPlan p = exact_plan(n, k);
    unsigned char *q = (unsigned char *)ws;
    auto take = [&](size_t bytes) {
        unsigned char *r = q;
        q += round256(bytes);
        return (void *)r;
    };
    const size_t win = (size_t)p.G * p.cap_win;
    ExactBufs b;
    b.lo_slot = (uint32_t *)take((size_t)p.G * p.cap_lo * 4);
    b.win_key = (uint32_t *)take(win * 4);
    b.win_ps = (uint64_t *)take(win * 8);
    b.ckey = (uint32_t *)take(win * 4);
    b.cps = (uint64_t *)take(win * 8);
    b.cnt_lo = (uint32_t *)take((size_t)p.G * 4);
    b.cnt_win = (uint32_t *)take((size_t)p.G * 4);
    b.x_slot = (uint32_t *)take((size_t)p.k * 4);
    b.ties = (uint64_t *)take((size_t)n * 8);
    b.st = (ExactState *)take(sizeof(ExactState));
    b.lo = p.lo;
    b.hi = p.hi;
    b.chunk = p.chunk;
    b.k = p.k;
    b.cap_lo = p.cap_lo;
    b.cap_win = p.cap_win;
    b.G = p.G;
    hipLaunchKernelGGL(k_exact_classify, dim3(p.G), dim3(256), 0, st, pid, n, seed, (uint32_t)step, b,
                       selected_out);
    hipLaunchKernelGGL(k_exact_select, dim3(1), dim3(SEL_T), 0, st, pid, n, seed, (uint32_t)step, b);
    if (dtype == PIC_F32)
        hipLaunchKernelGGL(k_exact_scatter<float>, dim3(p.G), dim3(256), 0, st, (float *)v, pid, n, b,
                           mass_ratio, seed, (uint32_t)step, selected_out);
    else
        hipLaunchKernelGGL(k_exact_scatter<double>, dim3(p.G), dim3(256), 0, st, (double *)v, pid, n, b,
                           mass_ratio, seed, (uint32_t)step, selected_out);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

int launch_recombine(int dtype, const RecombArgs &a, int num_cu, hipStream_t st)
{
    if (a.M <= 0) return PIC_OK;
    const int g = a.M < num_cu * 8 ? a.M : num_cu * 8;
    if (dtype == PIC_F32)
        hipLaunchKernelGGL(k_recombine<float>, dim3(g), dim3(RC_T), 0, st, a);
    else
        hipLaunchKernelGGL(k_recombine<double>, dim3(g), dim3(RC_T), 0, st, a);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}


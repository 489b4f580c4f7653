/*
 * oracle.c -- plain, slow, obviously correct FP64 CPU reference for the
 * electron collision step of a PIC-DSMC solver:
 *
 *   1. binning of particles into cells (Coulombic collision steps CCS1-CCS3),
 *   2. random pairing of the electrons of each cell (pairs of consecutive
 *      entries of the per-cell list, CCS3),
 *   3. the Takizuka & Abe (1977) binary Coulomb collision of every pair
 *      (CCS4-CCS5),
 *   4. the electron-neutral null-collision Monte Carlo step (DSMC collision
 *      kernel, paragraph "Null Collision Method"), run after the Coulomb
 *      step as in the operator split (PIC scheme table, S1 before S2a),
 *   5. per-cell moment sums and the optional momentum/energy correction.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library;
 * it shares no source, header, table or helper with it.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark load it.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (every
 * floating-point operation is rounded as written; no fused multiply-add).
 * OpenMP only splits the loop over cells; cells are independent and every
 * reduction runs in a fixed order, so results do not depend on the thread
 * count.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), key = (lo32(seed), hi32(seed)),
 * counter = (c0, lo32(step), domain, c3).  Domains used by the step:
 *   0  per particle, c0 = pid: word0 = pairing key, word1 = null-collision
 *      candidate draw, word2/word3 = Coulomb uniforms (see pair_collide)
 *   1  per null-collision candidate, c0 = pid: word0 = real/null test,
 *      word1 = polar cosine, word2 = azimuth
 *   2  per cell, c0 = cell id: judge-cell sampling of the learned gate
 *   3  per particle, c3 = replica: independent re-pairings for the label
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------ */
/* Philox4x32-10 from its published definition.                        */
/* ------------------------------------------------------------------ */
static const uint32_t PHILOX_M0 = 0xD2511F53u, PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u, PHILOX_W1 = 0xBB67AE85u;

void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }  /* key schedule */
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void draw(uint64_t seed, uint32_t c0, uint64_t step, uint32_t domain,
                 uint32_t c3, uint32_t w[4])
{
    uint32_t ctr[4] = {c0, (uint32_t)step, domain, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox(ctr, key, w);
}

/* Fill out[4*i .. 4*i+3] with Philox(c0[i], step, domain, c3). */
void orc_philox_fill(uint64_t seed, uint64_t step, uint32_t domain, uint32_t c3,
                     const uint32_t *c0, int64_t n, uint32_t *out)
{
    for (int64_t i = 0; i < n; ++i) draw(seed, c0[i], step, domain, c3, out + 4 * i);
}

/* Uniform in (0,1): ((x >> 9) + 1/2) * 2^-23, exactly representable in
 * binary32 and binary64; range [2^-24, 1 - 2^-24]. */
double orc_u01(uint32_t x) { return ((double)(x >> 9) + 0.5) * (1.0 / 8388608.0); }

/* ------------------------------------------------------------------ */
/* Binning: CCS1 (counts N_j), CCS2 (prefix sum -> I_j), CCS3 (place  */
/* each particle at I_j, I_j += 1).  Visiting particles in storage    */
/* order makes the placement a stable counting sort.                  */
/* ------------------------------------------------------------------ */
int orc_bin_cells(const int32_t *cell_of, int64_t n, int32_t n_cells,
                  int32_t *cell_start, int32_t *order)
{
    if (n < 0 || n_cells < 1) return 1;
    int64_t *count = calloc((size_t)n_cells, sizeof(int64_t));
    int64_t *next = malloc((size_t)n_cells * sizeof(int64_t));
    if (!count || !next) { free(count); free(next); return 4; }
    for (int64_t l = 0; l < n; ++l) {
        int32_t c = cell_of[l];
        if (c < 0 || c >= n_cells) { free(count); free(next); return 2; }
        count[c] += 1;
    }
    int64_t run = 0;
    for (int32_t j = 0; j < n_cells; ++j) {
        cell_start[j] = (int32_t)run;
        next[j] = run;
        run += count[j];
    }
    cell_start[n_cells] = (int32_t)run;
    for (int64_t l = 0; l < n; ++l) order[next[cell_of[l]]++] = (int32_t)l;
    free(count);
    free(next);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Pairing inside a cell.  The members of cell j are ordered by       */
/* (key, pid) with key = word0 of the particle's domain-0 draw; pairs */
/* are entries (2i, 2i+1) of that order; with an odd count the last   */
/* member has no partner this step.                                   */
/* ------------------------------------------------------------------ */
typedef struct { uint32_t key; uint32_t pid; int64_t slot; } member_t;

static int member_cmp(const void *a, const void *b)
{
    const member_t *x = a, *y = b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->pid != y->pid) return x->pid < y->pid ? -1 : 1;
    return 0;
}

/* Members of [lo, hi) sorted into S (slots), keyed with replica c3 of domain. */
static void order_members(const uint32_t *pid, int64_t lo, int64_t hi, uint64_t seed,
                          uint64_t step, uint32_t domain, uint32_t c3, member_t *S)
{
    for (int64_t m = lo; m < hi; ++m) {
        uint32_t w[4];
        draw(seed, pid[m], step, domain, c3, w);
        S[m - lo].key = w[0];
        S[m - lo].pid = pid[m];
        S[m - lo].slot = m;
    }
    qsort(S, (size_t)(hi - lo), sizeof(member_t), member_cmp);
}

/* sorted[cs[j] + r] = slot of the r-th member of cell j in pairing order;
 * partner[slot] = partner slot or -1 (idle). */
int orc_pairs(const int32_t *cell_start, const uint32_t *pid, int32_t n_cells,
              uint64_t seed, uint64_t step, int32_t *sorted, int32_t *partner)
{
    int64_t n = cell_start[n_cells];
    int64_t maxc = 0;
    for (int32_t j = 0; j < n_cells; ++j) {
        int64_t c = (int64_t)cell_start[j + 1] - cell_start[j];
        if (c < 0) return 1;
        if (c > maxc) maxc = c;
    }
    for (int64_t l = 0; l < n; ++l) partner[l] = -1;
    int err = 0;
#pragma omp parallel
    {
        member_t *S = malloc((size_t)(maxc > 0 ? maxc : 1) * sizeof(member_t));
        if (!S) {
#pragma omp atomic write
            err = 4;
        }
#pragma omp for schedule(dynamic, 1)
        for (int32_t j = 0; j < n_cells; ++j) {
            if (!S) continue;
            int64_t lo = cell_start[j], hi = cell_start[j + 1];
            order_members(pid, lo, hi, seed, step, 0u, 0u, S);
            for (int64_t r = 0; r < hi - lo; ++r) sorted[lo + r] = (int32_t)S[r].slot;
            for (int64_t i = 0; 2 * i + 1 < hi - lo; ++i) {
                partner[S[2 * i].slot] = (int32_t)S[2 * i + 1].slot;
                partner[S[2 * i + 1].slot] = (int32_t)S[2 * i].slot;
            }
        }
        free(S);
    }
    return err;
}

/* ------------------------------------------------------------------ */
/* Takizuka & Abe binary collision of one pair.                       */
/*                                                                    */
/* Code units: m_e = 1, (e^2 / 4 pi eps0)^2 = 1.  The tangent of half */
/* the scattering angle, delta, is Gaussian with variance             */
/*   s2 = 2 pi n lnL dt / (m_r^2 |u|^3),   m_r = 1/2 for e-e,          */
/* i.e. s2 = 8 pi n lnL dt / |u|^3.  delta = s * z with z standard    */
/* normal (Box-Muller, cosine branch, from U1, U2); the azimuth is    */
/* Phi = 2 pi U3.  The relative velocity u = v_a - v_b is rotated by  */
/* (Theta, Phi):                                                      */
/*   sin Theta = 2 delta / (1 + delta^2),                              */
/*   1 - cos Theta = 2 delta^2 / (1 + delta^2),                        */
/*   u' = u cos Theta + |u| sin Theta (cos Phi e1 + sin Phi e2)        */
/* with e1 = (ux uz, uy uz, -uperp^2) / (uperp |u|), e2 = (-uy, ux, 0)/uperp */
/* (and e1 = x, e2 = y when uperp = 0).  Each member receives half of */
/* the change with opposite signs, which conserves momentum exactly   */
/* and energy because |u'| = |u|.                                     */
/* ------------------------------------------------------------------ */
void orc_ta_delta(const double u[3], double s2, double U1, double U2, double U3,
                  double du[3])
{
    double ux = u[0], uy = u[1], uz = u[2];
    double uu = ux * ux + uy * uy + uz * uz;
    du[0] = du[1] = du[2] = 0.0;
    if (uu == 0.0) return;                     /* identical velocities: no-op */
    double umag = sqrt(uu);
    double uperp = sqrt(ux * ux + uy * uy);
    double z = sqrt(-2.0 * log(U1)) * cos(2.0 * ORC_PI * U2);
    double delta = sqrt(s2) * z;
    double sin_t = 2.0 * delta / (1.0 + delta * delta);
    double omc = 2.0 * delta * delta / (1.0 + delta * delta);
    double phi = 2.0 * ORC_PI * U3;
    double cphi = cos(phi), sphi = sin(phi);
    if (uperp > 0.0) {
        du[0] = (ux / uperp) * uz * sin_t * cphi - (uy / uperp) * umag * sin_t * sphi - ux * omc;
        du[1] = (uy / uperp) * uz * sin_t * cphi + (ux / uperp) * umag * sin_t * sphi - uy * omc;
        du[2] = -uperp * sin_t * cphi - uz * omc;
    } else {
        du[0] = umag * sin_t * cphi;
        du[1] = umag * sin_t * sphi;
        du[2] = -uz * omc;
    }
}

/* Variance of delta for a pair, code units. */
double orc_ta_s2(double uu_norm, double density, double lnL, double dt)
{
    return 8.0 * ORC_PI * density * lnL * dt / (uu_norm * uu_norm * uu_norm);
}

/* Collide the pair (a, b); uniforms come from the particles' domain-0 draws:
 * U1 = U(word2 of a), U2 = U(word3 of a), U3 = U(word2 of b). */
static void pair_collide(double *vx, double *vy, double *vz, int64_t a, int64_t b,
                         const uint32_t wa[4], const uint32_t wb[4], double density,
                         double lnL, double dt)
{
    double u[3] = {vx[a] - vx[b], vy[a] - vy[b], vz[a] - vz[b]};
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    if (uu == 0.0) return;
    double s2 = orc_ta_s2(sqrt(uu), density, lnL, dt);
    double du[3];
    orc_ta_delta(u, s2, orc_u01(wa[2]), orc_u01(wa[3]), orc_u01(wb[2]), du);
    double h0 = 0.5 * du[0], h1 = 0.5 * du[1], h2 = 0.5 * du[2];
    vx[a] += h0; vy[a] += h1; vz[a] += h2;
    vx[b] -= h0; vy[b] -= h1; vz[b] -= h2;
}

/* ------------------------------------------------------------------ */
/* Per-cell sums: count, momentum, twice the kinetic energy.          */
/* ------------------------------------------------------------------ */
static void cell_sums(const double *vx, const double *vy, const double *vz, int64_t lo,
                      int64_t hi, double S[5])
{
    S[0] = S[1] = S[2] = S[3] = S[4] = 0.0;
    for (int64_t m = lo; m < hi; ++m) {
        S[0] += 1.0;
        S[1] += vx[m];
        S[2] += vy[m];
        S[3] += vz[m];
        S[4] += vx[m] * vx[m] + vy[m] * vy[m] + vz[m] * vz[m];
    }
}

/* Correction restoring a cell's momentum and thermal energy to their values
 * before the Coulomb step: v <- V_old + alpha (v - V_new),
 * alpha = sqrt(E_th,old / E_th,new), E_th = sum|v|^2/2 - N |V|^2 / 2. */
static void conserve_cell(double *vx, double *vy, double *vz, int64_t lo, int64_t hi,
                          const double before[5])
{
    double after[5];
    cell_sums(vx, vy, vz, lo, hi, after);
    double N = before[0];
    if (N < 2.0) return;
    double Vo[3] = {before[1] / N, before[2] / N, before[3] / N};
    double Vn[3] = {after[1] / N, after[2] / N, after[3] / N};
    double Eo = 0.5 * before[4] - 0.5 * N * (Vo[0] * Vo[0] + Vo[1] * Vo[1] + Vo[2] * Vo[2]);
    double En = 0.5 * after[4] - 0.5 * N * (Vn[0] * Vn[0] + Vn[1] * Vn[1] + Vn[2] * Vn[2]);
    if (!(En > 0.0) || !(Eo >= 0.0)) return;
    double alpha = sqrt(Eo / En);
    for (int64_t m = lo; m < hi; ++m) {
        vx[m] = Vo[0] + alpha * (vx[m] - Vn[0]);
        vy[m] = Vo[1] + alpha * (vy[m] - Vn[1]);
        vz[m] = Vo[2] + alpha * (vz[m] - Vn[2]);
    }
}

/* ------------------------------------------------------------------ */
/* Null-collision Monte Carlo (elastic, isotropic).                   */
/*                                                                    */
/* Collision probability over dt: 1 - exp(-dt |v| sigma(E) n_n).  For */
/* sigma(E) = sigma0 E^-1/2 with E = |v|^2 / 2 the frequency          */
/* nu = n_n sigma0 |v| E^-1/2 = n_n sigma0 sqrt(2) is the same for    */
/* every speed, so the null-collision maximum nu_max equals it and    */
/* every candidate is a real collision.  A particle is a candidate    */
/* with probability P_null = 1 - exp(-nu_max dt): word1 of its        */
/* domain-0 draw below floor(P_null 2^32).  Candidates draw domain 1: */
/* real iff U(word0) nu_max < nu(E); new direction cos(theta) =       */
/* 1 - 2 U(word1), phi = 2 pi U(word2); elastic speed loss            */
/* |v'|^2 = |v|^2 (1 - 2 (m/M) (1 - vhat . s)).                        */
/* ------------------------------------------------------------------ */
uint64_t orc_mcc_threshold(double dt, double sigma0, double n_neutral)
{
    double nu_max = n_neutral * sigma0 * sqrt(2.0);
    double p = 1.0 - exp(-nu_max * dt);
    double t = floor(p * 4294967296.0);
    if (t < 0.0) t = 0.0;
    if (t > 4294967296.0) t = 4294967296.0;
    return (uint64_t)t;
}

static void mcc_particle(double *vx, double *vy, double *vz, int64_t l, uint32_t pid,
                         uint32_t w1_candidate, uint64_t thr, double nu_max, double nu_E,
                         double mass_ratio, uint64_t seed, uint64_t step,
                         uint8_t *flag_out)
{
    int cand = (uint64_t)w1_candidate < thr;
    if (flag_out) flag_out[l] = (uint8_t)cand;
    if (!cand) return;
    uint32_t w[4];
    draw(seed, pid, step, 1u, 0u, w);
    if (!(orc_u01(w[0]) * nu_max < nu_E)) return;  /* null collision */
    double ct = 1.0 - 2.0 * orc_u01(w[1]);
    double st = sqrt(1.0 - ct * ct);
    double ph = 2.0 * ORC_PI * orc_u01(w[2]);
    double s[3] = {st * cos(ph), st * sin(ph), ct};
    double sp2 = vx[l] * vx[l] + vy[l] * vy[l] + vz[l] * vz[l];
    double sp = sqrt(sp2);
    double scale = sp;
    if (sp > 0.0 && mass_ratio != 0.0) {
        double cosx = (vx[l] * s[0] + vy[l] * s[1] + vz[l] * s[2]) / sp;
        scale = sp * sqrt(1.0 - 2.0 * mass_ratio * (1.0 - cosx));
    }
    vx[l] = scale * s[0];
    vy[l] = scale * s[1];
    vz[l] = scale * s[2];
}

/* Stand-alone null-collision step over n particles (storage order irrelevant). */
int orc_mcc(double *v, const uint32_t *pid, int64_t n, double dt, double sigma0,
            double n_neutral, double mass_ratio, uint64_t seed, uint64_t step,
            uint8_t *candidate_out)
{
    if (n < 0 || !(dt > 0.0)) return 1;
    double *vx = v, *vy = v + n, *vz = v + 2 * n;
    uint64_t thr = orc_mcc_threshold(dt, sigma0, n_neutral);
    double nu_max = n_neutral * sigma0 * sqrt(2.0);
#pragma omp parallel for schedule(static)
    for (int64_t l = 0; l < n; ++l) {
        uint32_t w[4];
        draw(seed, pid[l], step, 0u, 0u, w);
        mcc_particle(vx, vy, vz, l, pid[l], w[1], thr, nu_max, nu_max, mass_ratio, seed,
                     step, candidate_out);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* One full step.                                                      */
/* ------------------------------------------------------------------ */
typedef struct {
    double dt;              /* time step (> 0) */
    double lnL;             /* Coulomb logarithm (> 0) */
    const double *density;  /* per-cell electron density, NULL => 1 */
    uint64_t seed;
    uint64_t step;          /* low 32 bits enter the counter */
    int32_t conserve;       /* apply the per-cell conservation correction */
    int32_t mcc;            /* run the null-collision step after Coulomb */
    double sigma0, n_neutral, mass_ratio;
    const double *dt_scale; /* per-cell multiplier of dt for Coulomb, NULL => 1 */
    const uint8_t *skip;    /* per-cell: nonzero => no Coulomb collision */
} orc_params;

/* v = [vx(n) | vy(n) | vz(n)].  Storage (v, pid, cell_of) is first
 * permuted into stable cell order; cell_start (M+1) is returned if non-NULL. */
int orc_step(double *v, int32_t *cell_of, uint32_t *pid, int64_t n, int32_t n_cells,
             const orc_params *p, int32_t *cell_start_out)
{
    if (n < 0 || n_cells < 1 || !(p->dt > 0.0) || !(p->lnL > 0.0)) return 1;
    int32_t *cs = malloc((size_t)(n_cells + 1) * sizeof(int32_t));
    int32_t *order = malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    double *tmp = malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    int32_t *itmp = malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!cs || !order || !tmp || !itmp) {
        free(cs); free(order); free(tmp); free(itmp);
        return 4;
    }
    int rc = orc_bin_cells(cell_of, n, n_cells, cs, order);
    if (rc) { free(cs); free(order); free(tmp); free(itmp); return rc; }
    /* permute storage into cell order */
    for (int c = 0; c < 3; ++c) {
        double *comp = v + (int64_t)c * n;
        for (int64_t k = 0; k < n; ++k) tmp[k] = comp[order[k]];
        memcpy(comp, tmp, (size_t)n * sizeof(double));
    }
    for (int64_t k = 0; k < n; ++k) itmp[k] = (int32_t)pid[order[k]];
    memcpy(pid, itmp, (size_t)n * sizeof(uint32_t));
    for (int64_t k = 0; k < n; ++k) itmp[k] = cell_of[order[k]];
    memcpy(cell_of, itmp, (size_t)n * sizeof(int32_t));
    free(tmp);
    free(itmp);

    double *vx = v, *vy = v + n, *vz = v + 2 * n;
    int64_t maxc = 0;
    for (int32_t j = 0; j < n_cells; ++j)
        if (cs[j + 1] - cs[j] > maxc) maxc = cs[j + 1] - cs[j];
    uint64_t thr = orc_mcc_threshold(p->dt, p->sigma0, p->n_neutral);
    double nu_max = p->n_neutral * p->sigma0 * sqrt(2.0);
    int err = 0;
#pragma omp parallel
    {
        member_t *S = malloc((size_t)(maxc > 0 ? maxc : 1) * sizeof(member_t));
        if (!S) {
#pragma omp atomic write
            err = 4;
        }
#pragma omp for schedule(dynamic, 1)
        for (int32_t j = 0; j < n_cells; ++j) {
            if (!S) continue;
            int64_t lo = cs[j], hi = cs[j + 1];
            double before[5];
            cell_sums(vx, vy, vz, lo, hi, before);
            int skip = p->skip ? (p->skip[j] != 0) : 0;
            if (!skip) {
                double dens = p->density ? p->density[j] : 1.0;
                double dtc = p->dt * (p->dt_scale ? p->dt_scale[j] : 1.0);
                order_members(pid, lo, hi, p->seed, p->step, 0u, 0u, S);
                for (int64_t i = 0; 2 * i + 1 < hi - lo; ++i) {
                    int64_t a = S[2 * i].slot, b = S[2 * i + 1].slot;
                    uint32_t wa[4], wb[4];
                    draw(p->seed, pid[a], p->step, 0u, 0u, wa);
                    draw(p->seed, pid[b], p->step, 0u, 0u, wb);
                    pair_collide(vx, vy, vz, a, b, wa, wb, dens, p->lnL, dtc);
                }
                if (p->conserve) conserve_cell(vx, vy, vz, lo, hi, before);
            }
            if (p->mcc) {
                for (int64_t m = lo; m < hi; ++m) {
                    uint32_t w[4];
                    draw(p->seed, pid[m], p->step, 0u, 0u, w);
                    mcc_particle(vx, vy, vz, m, pid[m], w[1], thr, nu_max, nu_max,
                                 p->mass_ratio, p->seed, p->step, NULL);
                }
            }
        }
        free(S);
    }
    if (cell_start_out) memcpy(cell_start_out, cs, (size_t)(n_cells + 1) * sizeof(int32_t));
    free(cs);
    free(order);
    return err;
}

/* Apply the correction to every cell given the sums taken before the
 * collision (before[5*j .. 5*j+4] = N, sum vx, sum vy, sum vz, sum |v|^2). */
int orc_conserve_cells(double *v, int64_t n, const int32_t *cell_start, int32_t n_cells,
                       const double *before)
{
    double *vx = v, *vy = v + n, *vz = v + 2 * n;
    for (int32_t j = 0; j < n_cells; ++j)
        conserve_cell(vx, vy, vz, cell_start[j], cell_start[j + 1], before + 5 * (int64_t)j);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Per-cell raw moment sums over the members [cs[j], cs[j+1]):         */
/*  0 N, 1-3 sum v, 4-6 sum vx^2, vy^2, vz^2, 7-9 sum vx vy, vx vz,    */
/*  vy vz, 10-12 sum |v|^2 v, 13 sum |v|^4.                            */
/* ------------------------------------------------------------------ */
int orc_cell_moments(const double *v, int64_t n, const int32_t *cell_start, int32_t n_cells,
                     double *out)
{
    const double *vx = v, *vy = v + n, *vz = v + 2 * n;
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < n_cells; ++j) {
        double *o = out + 14 * (int64_t)j;
        for (int k = 0; k < 14; ++k) o[k] = 0.0;
        for (int64_t m = cell_start[j]; m < cell_start[j + 1]; ++m) {
            double x = vx[m], y = vy[m], z = vz[m];
            double q = x * x + y * y + z * z;
            o[0] += 1.0;
            o[1] += x; o[2] += y; o[3] += z;
            o[4] += x * x; o[5] += y * y; o[6] += z * z;
            o[7] += x * y; o[8] += x * z; o[9] += y * z;
            o[10] += q * x; o[11] += q * y; o[12] += q * z;
            o[13] += q * q;
        }
    }
    return 0;
}

/* Relative-velocity list of one pairing of every cell (label support):
 * replica c3 of domain 3 keys a fresh pairing; for pair i of cell j,
 * out_u[3*k..] = u and out_cell[k] = j, k counting pairs globally in cell
 * order.  Returns the number of pairs written (<= n/2). */
int64_t orc_repair_u(const double *v, int64_t n, const int32_t *cell_start, int32_t n_cells,
                     const uint32_t *pid, uint64_t seed, uint64_t step, uint32_t replica,
                     double *out_u, int32_t *out_cell)
{
    const double *vx = v, *vy = v + n, *vz = v + 2 * n;
    int64_t maxc = 0;
    for (int32_t j = 0; j < n_cells; ++j)
        if (cell_start[j + 1] - cell_start[j] > maxc) maxc = cell_start[j + 1] - cell_start[j];
    member_t *S = malloc((size_t)(maxc > 0 ? maxc : 1) * sizeof(member_t));
    if (!S) return -1;
    int64_t k = 0;
    for (int32_t j = 0; j < n_cells; ++j) {
        int64_t lo = cell_start[j], hi = cell_start[j + 1];
        order_members(pid, lo, hi, seed, step, 3u, replica, S);
        for (int64_t i = 0; 2 * i + 1 < hi - lo; ++i) {
            int64_t a = S[2 * i].slot, b = S[2 * i + 1].slot;
            out_u[3 * k + 0] = vx[a] - vx[b];
            out_u[3 * k + 1] = vy[a] - vy[b];
            out_u[3 * k + 2] = vz[a] - vz[b];
            out_cell[k] = j;
            ++k;
        }
    }
    free(S);
    return k;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* DSMC-Coll step for electron-heavy collisions C1..C4 (Table          */
/* "DSMC Collision Step", CS0-CS5, and the probability formula of the */
/* section "DSMC Collision Kernel"):                                  */
/*   pi_c = 1 - exp(-dt |v| sigma_c(E) n_k(c)),  E = |v|^2 / 2,        */
/* C1 elastic and C2 ionization and C3 excitation on the ground-state */
/* density n_g, C4 two-step ionization on the metastable density n_m. */
/* sigma_c: piecewise cubic in E on breakpoints e_0 = 0 < ... < e_P   */
/* (constant beyond e_P), clipped at 0, zero below the threshold.     */
/* Selection (reading): U(w0) of the domain-6 draw picks the first    */
/* channel whose cumulative probability exceeds it.  Post-collision   */
/* (Vahedi & Surendra): direction cos = 1 - 2 U(w1), phi = 2 pi U(w2); */
/* elastic keeps |v| up to the m/M loss; excitation loses eps_3;      */
/* ionization loses eps_c and splits the rest as U(w3) : 1 - U(w3)    */
/* between the scattered and a new electron, whose direction comes    */
/* from words 1, 2 of the domain-7 draw.  The new electron gets pid   */
/* pid_base + pid and the parent's cell, appended at *count.          */
/* ------------------------------------------------------------------ */
double orc_dsmc_sigma(int32_t c, double E, int32_t nseg, const double *breaks,
                      const double *coef, const double *thr)
{
    if (E < thr[c]) return 0.0;
    int32_t p = 0;
    while (p + 1 < nseg && E >= breaks[p + 1]) ++p;
    double t = E - breaks[p];
    const double tmax = breaks[p + 1] - breaks[p];
    if (t > tmax) t = tmax;   /* beyond the last breakpoint */
    const double *a = coef + ((size_t)c * nseg + p) * 4;
    double s = ((a[3] * t + a[2]) * t + a[1]) * t + a[0];
    return s > 0.0 ? s : 0.0;
}

static void iso_dir(uint32_t wa, uint32_t wb, double s[3])
{
    double ct = 1.0 - 2.0 * orc_u01(wa);
    double st = sqrt(fmax(0.0, 1.0 - ct * ct));
    double ph = 2.0 * ORC_PI * orc_u01(wb);
    s[0] = st * cos(ph);
    s[1] = st * sin(ph);
    s[2] = ct;
}

int orc_dsmc(double *v, int64_t n, const int32_t *cell, const uint32_t *pid, const double *ng,
             const double *nm, double ng0, double nm0, double dt, int32_t nseg,
             const double *breaks, const double *coef, const double *thr, double mass_ratio,
             uint64_t seed, uint64_t step, uint32_t pid_base, double *v_new, int64_t cap,
             uint32_t *pid_new, int32_t *cell_new, int64_t *count, uint8_t *chan_out)
{
    double *vx = v, *vy = v + n, *vz = v + 2 * n;
    for (int64_t l = 0; l < n; ++l) {
        const double x = vx[l], y = vy[l], z = vz[l];
        const double sp2 = x * x + y * y + z * z;
        const double sp = sqrt(sp2);
        const double E = 0.5 * sp2;
        const double dg = ng ? ng[cell[l]] : ng0;
        const double dm = nm ? nm[cell[l]] : nm0;
        uint32_t w[4];
        draw(seed, pid[l], step, 6u, 0u, w);
        const double R0 = orc_u01(w[0]);
        double cum = 0.0;
        int32_t ch = -1;
        for (int32_t c = 0; c < 4 && ch < 0; ++c) {
            const double dens = c == 3 ? dm : dg;
            const double pc = 1.0 - exp(-dt * sp * orc_dsmc_sigma(c, E, nseg, breaks, coef, thr) * dens);
            cum += pc;
            if (R0 < cum) ch = c;
        }
        if (chan_out) chan_out[l] = (uint8_t)(ch + 1);
        if (ch < 0) continue;
        double s[3];
        iso_dir(w[1], w[2], s);
        double scale;
        if (ch == 0) {
            scale = sp;
            if (sp > 0.0 && mass_ratio != 0.0) {
                const double cosx = (x * s[0] + y * s[1] + z * s[2]) / sp;
                scale = sp * sqrt(1.0 - 2.0 * mass_ratio * (1.0 - cosx));
            }
        } else if (ch == 2) {
            scale = sqrt(2.0 * (E - thr[2]));
        } else {
            const double rem = E - thr[ch];
            const double e1 = orc_u01(w[3]) * rem;
            const double e2 = rem - e1;
            scale = sqrt(2.0 * e1);
            uint32_t w2[4];
            draw(seed, pid[l], step, 7u, 0u, w2);
            double s2[3];
            iso_dir(w2[1], w2[2], s2);
            const double sc2 = sqrt(2.0 * e2);
            const int64_t k = (*count)++;
            if (k < cap) {
                v_new[k] = sc2 * s2[0];
                v_new[cap + k] = sc2 * s2[1];
                v_new[2 * cap + k] = sc2 * s2[2];
                pid_new[k] = pid_base + pid[l];
                cell_new[k] = cell[l];
            }
        }
        vx[l] = scale * s[0];
        vy[l] = scale * s[1];
        vz[l] = scale * s[2];
    }
    return *count > cap ? 1 : 0;
}

/* ------------------------------------------------------------------ */
/* Exact-count null-collision selection (the paper picks P_null N      */
/* particles at random): K = round(P_null n) particles, those with the */
/* K smallest candidate words (word 1 of the domain-0 draw, the word   */
/* the per-particle test compares with floor(P_null 2^32)), equal     */
/* words ordered by pid, then slot -- a uniformly random K-subset.     */
/* Each selected particle scatters as in orc_mcc (domain 1).           */
/* ------------------------------------------------------------------ */
typedef struct {
    uint32_t key, pid;
    int64_t slot;
} sel_t;

static int sel_cmp(const void *a, const void *b)
{
    const sel_t *x = a, *y = b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->pid != y->pid) return x->pid < y->pid ? -1 : 1;
    return x->slot < y->slot ? -1 : x->slot > y->slot;
}

int64_t orc_mcc_exact_count(int64_t n, double dt, double sigma0, double n_neutral)
{
    const double nu_max = n_neutral * sigma0 * sqrt(2.0);
    const double p = 1.0 - exp(-nu_max * dt);
    return (int64_t)llround(p * (double)n);
}

int orc_mcc_exact(double *v, const uint32_t *pid, int64_t n, double dt, double sigma0,
                  double n_neutral, double mass_ratio, uint64_t seed, uint64_t step,
                  uint8_t *selected_out)
{
    if (n < 0 || !(dt > 0.0)) return 1;
    const int64_t K = orc_mcc_exact_count(n, dt, sigma0, n_neutral);
    sel_t *s = malloc((size_t)(n > 0 ? n : 1) * sizeof(sel_t));
    if (!s) return 2;
    for (int64_t l = 0; l < n; ++l) {
        uint32_t w[4];
        draw(seed, pid[l], step, 0u, 0u, w);
        s[l].key = w[1];
        s[l].pid = pid[l];
        s[l].slot = l;
    }
    qsort(s, (size_t)n, sizeof(sel_t), sel_cmp);
    double *vx = v, *vy = v + n, *vz = v + 2 * n;
    const double nu_max = n_neutral * sigma0 * sqrt(2.0);
    if (selected_out) memset(selected_out, 0, (size_t)n);
    for (int64_t k = 0; k < K && k < n; ++k) {
        const int64_t l = s[k].slot;
        /* every selected particle is a candidate: threshold 2^32 */
        mcc_particle(vx, vy, vz, l, pid[l], 0u, (uint64_t)1 << 32, nu_max, nu_max, mass_ratio,
                     seed, step, selected_out);
    }
    free(s);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Particle-to-cell sums (section "Particle-to-Cell"): the sum of the  */
/* per-particle vector V_l over the particles of each cell,            */
/* out[j nq + k] = sum_{l : cell_of[l] = j} q[k n + l], in particle    */
/* order.  Ids outside [0, M) are skipped; the return value counts     */
/* them.                                                               */
/* ------------------------------------------------------------------ */
int64_t orc_p2c(const double *q, int32_t nq, const int32_t *cell_of, int64_t n, int32_t M,
                double *out)
{
    int64_t bad = 0;
    for (int64_t j = 0; j < (int64_t)M * nq; ++j) out[j] = 0.0;
    for (int64_t l = 0; l < n; ++l) {
        const int32_t c = cell_of[l];
        if (c < 0 || c >= M) {
            ++bad;
            continue;
        }
        for (int32_t k = 0; k < nq; ++k) out[(int64_t)c * nq + k] += q[(int64_t)k * n + l];
    }
    return bad;
}

/* ------------------------------------------------------------------ */
/* Recombination C5 (section "Kernel for Recombination Collision C5"): */
/* in each cell the primaries (flag set, weight > 0) are matched one   */
/* to one with catalytes (flag clear, weight > 0).  Reading of the     */
/* atomic pop: catalytes are taken in storage order from a per-cell    */
/* offset o_j = floor(word0 C_j / 2^32) (domain 9 draw on the cell     */
/* index), wrapping: the k-th primary in storage order gets the        */
/* catalyte of rank (o_j + k) mod C_j, for k < min(P_j, C_j).  The     */
/* catalyte takes the primary's kinetic energy plus the released       */
/* energy eps (|v|^2 / 2 units) in an isotropic direction (words 1, 2  */
/* of a domain 8 draw on its pid); the primary's weight becomes 0.     */
/* Storage in cell order, cell_start of M + 1 entries.  events[j]      */
/* (nullable) receives the number of recombinations in cell j.         */
/* ------------------------------------------------------------------ */
int orc_recombine(double *v, double *w, const uint32_t *pid, const uint8_t *primary, int64_t n,
                  const int32_t *cell_start, int32_t M, double eps, uint64_t seed, uint64_t step,
                  int32_t *events)
{
    double *vx = v, *vy = v + n, *vz = v + 2 * n;
    int64_t *prim = malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *cat = malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!prim || !cat) {
        free(prim);
        free(cat);
        return 2;
    }
    for (int32_t j = 0; j < M; ++j) {
        int64_t P = 0, C = 0;
        for (int64_t l = cell_start[j]; l < cell_start[j + 1]; ++l) {
            if (!(w[l] > 0.0)) continue;
            if (primary[l]) prim[P++] = l;
            else cat[C++] = l;
        }
        const int64_t m = P < C ? P : C;
        if (events) events[j] = (int32_t)m;
        if (m == 0) continue;
        uint32_t cw[4];
        draw(seed, (uint32_t)j, step, 9u, 0u, cw);
        const int64_t o = (int64_t)(((uint64_t)cw[0] * (uint64_t)C) >> 32);
        for (int64_t k = 0; k < m; ++k) {
            const int64_t p = prim[k], c = cat[(o + k) % C];
            const double ep = 0.5 * (vx[p] * vx[p] + vy[p] * vy[p] + vz[p] * vz[p]);
            const double ec = 0.5 * (vx[c] * vx[c] + vy[c] * vy[c] + vz[c] * vz[c]);
            const double sp = sqrt(2.0 * (ec + ep + eps));
            uint32_t dw[4];
            double s[3];
            draw(seed, pid[c], step, 8u, 0u, dw);
            iso_dir(dw[1], dw[2], s);
            vx[c] = sp * s[0];
            vy[c] = sp * s[1];
            vz[c] = sp * s[2];
            w[p] = 0.0;
        }
    }
    free(prim);
    free(cat);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Nanbu's Coulomb operator (the alternative to Takizuka & Abe the    */
/* paper names in its related work).  Same pairs as the T&A step; the */
/* pair (a, b), a the lower slot, turns its relative velocity by an   */
/* angle chi whose cosine has density proportional to exp(A cos chi), */
/* A solving coth A - 1/A = exp(-s), so that <cos chi> = exp(-s).      */
/* Reading: s = 2 s2 with s2 the T&A variance of tan(Theta/2), so both */
/* operators have the same small-angle diffusion (<chi^2> ~ 2 s).      */
/* cos chi by inversion of its distribution with U = U(word 2 of a);  */
/* azimuth 2 pi U(word 2 of b); rotation and halves as in T&A.         */
/* ------------------------------------------------------------------ */
/* Langevin function coth A - 1/A and its derivative (series below 0.1). */
static void langevin(double A, double *L, double *dL)
{
    if (A < 0.1) {
        double A2 = A * A;
        *L = A * (1.0 / 3.0 - A2 * (1.0 / 45.0 - A2 * (2.0 / 945.0 - A2 / 4725.0)));
        *dL = 1.0 / 3.0 - A2 * (1.0 / 15.0 - A2 * (2.0 / 189.0 - A2 / 675.0));
    } else {   /* t = exp(-2A): coth A = (1 + t)/(1 - t), 1/sinh^2 A = 4t/(1 - t)^2 */
        double t = exp(-2.0 * A), d = 1.0 - t;
        *L = (1.0 + t) / d - 1.0 / A;
        *dL = 1.0 / (A * A) - 4.0 * t / (d * d);
    }
}

double orc_nanbu_A(double s)
{
    if (s <= 0.01) return -1.0 / expm1(-s);       /* coth A = 1 to double precision */
    double y = exp(-s);
    if (s > 11.5) return 3.0 * y;                 /* L(A) = A/3 to 1e-10 */
    double A = y * (3.0 - y * y) / (1.0 - y * y); /* approximate inverse, then Newton */
    for (int it = 0; it < 4; ++it) {   /* from within 2%: quadratic convergence */
        double L, dL;
        langevin(A, &L, &dL);
        A -= (L - y) / dL;
    }
    return A;
}

/* 1 - cos chi for the uniform U: -log(U + (1 - U) exp(-2A)) / A, the
 * argument written 1 - q with q = (1 - U)(1 - exp(-2A)) while q < 1/2 (log1p
 * of -q), and as the sum itself otherwise (no cancellation when U and
 * exp(-2A) are both small). */
double orc_nanbu_omc(double A, double U)
{
    if (!(A > 1e-300)) return 2.0 * (1.0 - U);    /* isotropic */
    double q = (1.0 - U) * -expm1(-2.0 * A);
    double omc = q < 0.5 ? -log1p(-q) / A : -log(U + (1.0 - U) * exp(-2.0 * A)) / A;
    return omc < 2.0 ? omc : 2.0;
}

int orc_nanbu(double *v, int64_t n, const int32_t *cell_start, const uint32_t *pid, int32_t M,
              double dt, double lnL, const double *density, uint64_t seed, uint64_t step)
{
    if (cell_start[M] != n) return 1;
    int32_t *sorted = malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int32_t *partner = malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!sorted || !partner) {
        free(sorted);
        free(partner);
        return 2;
    }
    int rc = orc_pairs(cell_start, pid, M, seed, step, sorted, partner);
    double *vx = v, *vy = v + n, *vz = v + 2 * n;
    for (int32_t j = 0; j < M && !rc; ++j) {
        double dens = density ? density[j] : 1.0;
        for (int64_t a = cell_start[j]; a < cell_start[j + 1]; ++a) {
            int64_t b = partner[a];
            if (b <= a) continue;
            double u[3] = {vx[a] - vx[b], vy[a] - vy[b], vz[a] - vz[b]};
            double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
            if (uu == 0.0) continue;
            double um = sqrt(uu), uperp = sqrt(u[0] * u[0] + u[1] * u[1]);
            double s = 2.0 * orc_ta_s2(um, dens, lnL, dt);
            uint32_t wa[4], wb[4];
            draw(seed, pid[a], step, 0u, 0u, wa);
            draw(seed, pid[b], step, 0u, 0u, wb);
            double omc = orc_nanbu_omc(orc_nanbu_A(s), orc_u01(wa[2]));
            double sin_t = sqrt(omc * (2.0 - omc));
            double phi = 2.0 * ORC_PI * orc_u01(wb[2]);
            double cphi = cos(phi), sphi = sin(phi), du[3];
            if (uperp > 0.0) {
                du[0] = (u[0] / uperp) * u[2] * sin_t * cphi - (u[1] / uperp) * um * sin_t * sphi - u[0] * omc;
                du[1] = (u[1] / uperp) * u[2] * sin_t * cphi + (u[0] / uperp) * um * sin_t * sphi - u[1] * omc;
                du[2] = -uperp * sin_t * cphi - u[2] * omc;
            } else {
                du[0] = um * sin_t * cphi;
                du[1] = um * sin_t * sphi;
                du[2] = -u[2] * omc;
            }
            double h0 = 0.5 * du[0], h1 = 0.5 * du[1], h2 = 0.5 * du[2];
            vx[a] += h0; vy[a] += h1; vz[a] += h2;
            vx[b] -= h0; vy[b] -= h1; vz[b] -= h2;
        }
    }
    free(sorted);
    free(partner);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Takizuka & Abe step with their triplet for odd cells (the paper    */
/* leaves the last member of an odd cell idle).  Pairs as in          */
/* orc_pairs; in a cell of odd N >= 3 the last three members in       */
/* pairing order, p0 p1 p2, collide pairwise at dt/2 in the order     */
/* (p0, p1), (p1, p2), (p2, p0), each on the velocities the previous   */
/* one left.  Uniforms: (p0, p1) as a regular pair (domain 0 of p0 and */
/* p1); (p1, p2) from domain 4 draws of p1 and p2; (p2, p0) from      */
/* domain 5 draws of p2 and p0.  Storage in cell order.               */
/* ------------------------------------------------------------------ */
int orc_step_triplet(double *v, int64_t n, const int32_t *cell_start, const uint32_t *pid, int32_t M,
                     double dt, double lnL, const double *density, uint64_t seed, uint64_t step)
{
    if (cell_start[M] != n) return 1;
    int32_t *sorted = malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int32_t *partner = malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!sorted || !partner) {
        free(sorted);
        free(partner);
        return 2;
    }
    int rc = orc_pairs(cell_start, pid, M, seed, step, sorted, partner);
    double *vx = v, *vy = v + n, *vz = v + 2 * n;
    for (int32_t j = 0; j < M && !rc; ++j) {
        const double dens = density ? density[j] : 1.0;
        const int64_t lo = cell_start[j], N = (int64_t)cell_start[j + 1] - lo;
        const int64_t tri = (N % 2 == 1 && N >= 3) ? N - 3 : N;   /* first triplet position */
        for (int64_t r = 0; r + 1 < tri; r += 2) {
            const int64_t a = sorted[lo + r], b = sorted[lo + r + 1];
            uint32_t wa[4], wb[4];
            draw(seed, pid[a], step, 0u, 0u, wa);
            draw(seed, pid[b], step, 0u, 0u, wb);
            pair_collide(vx, vy, vz, a, b, wa, wb, dens, lnL, dt);
        }
        if (tri < N) {
            const int64_t p[3] = {sorted[lo + tri], sorted[lo + tri + 1], sorted[lo + tri + 2]};
            const uint32_t dom[3] = {0u, 4u, 5u};
            for (int c = 0; c < 3; ++c) {
                const int64_t a = p[c], b = p[(c + 1) % 3];
                uint32_t wa[4], wb[4];
                draw(seed, pid[a], step, dom[c], 0u, wa);
                draw(seed, pid[b], step, dom[c], 0u, wb);
                pair_collide(vx, vy, vz, a, b, wa, wb, dens, lnL, 0.5 * dt);
            }
        }
    }
    free(sorted);
    free(partner);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Variable-weight particles (the paper names weights that differ     */
/* between particles as the next step beyond its uniform weights,      */
/* Sec. "Conclusion").  Reading W1, after Nanbu & Yonemura's rule for  */
/* binary collisions of weighted particles: the pairs, deflection and  */
/* half change h = du/2 are the uniform step's (s^2 from the cell      */
/* density); then the member of smaller weight w_l takes its half       */
/* change always and the one of larger weight w_h with probability     */
/* w_l / w_h: accepted iff U4 * w_h < w_l in binary64, with U4 the      */
/* uniform of word 3 of the second member's domain-0 draw (the one word */
/* of the pair's two draws the uniform step leaves unused).  Equal      */
/* weights: both take it (the uniform step).  For w_a >= w_b the        */
/* expected weighted change of momentum, w_a (w_b/w_a) h - w_b h, is   */
/* zero, and so is that of w |v|^2 since u.h = -|h|^2: both are         */
/* conserved on average, not in each collision.  Null collisions as in */
/* the uniform step.  Storage in cell order.                            */
/* ------------------------------------------------------------------ */
int orc_step_weighted(double *v, const double *w, int64_t n, const int32_t *cell_start,
                      const uint32_t *pid, int32_t M, double dt, double lnL, const double *density,
                      uint64_t seed, uint64_t step, int32_t mcc, double sigma0, double n_neutral,
                      double mass_ratio)
{
    if (cell_start[M] != n) return 1;
    int32_t *sorted = malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int32_t *partner = malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!sorted || !partner) {
        free(sorted);
        free(partner);
        return 2;
    }
    int rc = orc_pairs(cell_start, pid, M, seed, step, sorted, partner);
    double *vx = v, *vy = v + n, *vz = v + 2 * n;
    const uint64_t thr = orc_mcc_threshold(dt, sigma0, n_neutral);
    const double nu_max = n_neutral * sigma0 * sqrt(2.0);
    for (int32_t j = 0; j < M && !rc; ++j) {
        const double dens = density ? density[j] : 1.0;
        const int64_t lo = cell_start[j], N = (int64_t)cell_start[j + 1] - lo;
        for (int64_t r = 0; r + 1 < N; r += 2) {
            const int64_t a = sorted[lo + r], b = sorted[lo + r + 1];
            uint32_t wa[4], wb[4];
            draw(seed, pid[a], step, 0u, 0u, wa);
            draw(seed, pid[b], step, 0u, 0u, wb);
            double u[3] = {vx[a] - vx[b], vy[a] - vy[b], vz[a] - vz[b]};
            double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
            if (uu == 0.0) continue;
            double du[3];
            orc_ta_delta(u, orc_ta_s2(sqrt(uu), dens, lnL, dt), orc_u01(wa[2]), orc_u01(wa[3]),
                         orc_u01(wb[2]), du);
            double h0 = 0.5 * du[0], h1 = 0.5 * du[1], h2 = 0.5 * du[2];
            int take_a = 1, take_b = 1;
            if (w[a] != w[b]) {
                const double U4 = orc_u01(wb[3]);
                if (w[a] > w[b]) take_a = U4 * w[a] < w[b];
                else take_b = U4 * w[b] < w[a];
            }
            if (take_a) { vx[a] += h0; vy[a] += h1; vz[a] += h2; }
            if (take_b) { vx[b] -= h0; vy[b] -= h1; vz[b] -= h2; }
        }
        if (mcc) {
            for (int64_t m = lo; m < lo + N; ++m) {
                uint32_t d0[4];
                draw(seed, pid[m], step, 0u, 0u, d0);
                mcc_particle(vx, vy, vz, m, pid[m], d0[1], thr, nu_max, nu_max, mass_ratio, seed,
                             step, NULL);
            }
        }
    }
    free(sorted);
    free(partner);
    return rc;
}

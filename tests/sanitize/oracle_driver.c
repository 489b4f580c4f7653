/* Runs every entry point of the oracle once on small random inputs, for the
 * address and undefined-behaviour sanitizer build of oracle.c (the oracle is
 * test infrastructure; this driver is part of its tests).  Exit 0 when every
 * call returns its success code. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double dt, lnL;
    const double *density;
    uint64_t seed, step;
    int32_t conserve, mcc;
    double sigma0, n_neutral, mass_ratio;
    const double *dt_scale;
    const uint8_t *skip;
} orc_params;

int orc_step(double *v, int32_t *cell_of, uint32_t *pid, int64_t n, int32_t n_cells,
             const orc_params *p, int32_t *cell_start_out);
int orc_pairs(const int32_t *cell_start, const uint32_t *pid, int32_t n_cells, uint64_t seed,
              uint64_t step, int32_t *sorted, int32_t *partner);
int orc_cell_moments(const double *v, int64_t n, const int32_t *cell_start, int32_t n_cells,
                     double *out);
int orc_mcc(double *v, const uint32_t *pid, int64_t n, double dt, double sigma0, double n_neutral,
            double mass_ratio, uint64_t seed, uint64_t step, uint8_t *cand_out);
int orc_mcc_exact(double *v, const uint32_t *pid, int64_t n, double dt, double sigma0,
                  double n_neutral, double mass_ratio, uint64_t seed, uint64_t step,
                  uint8_t *selected_out);
int64_t orc_p2c(const double *q, int32_t nq, const int32_t *cell_of, int64_t n, int32_t M,
                double *out);
int orc_recombine(double *v, double *w, const uint32_t *pid, const uint8_t *primary, int64_t n,
                  const int32_t *cell_start, int32_t M, double eps, uint64_t seed, uint64_t step,
                  int32_t *events);
int orc_nanbu(double *v, int64_t n, const int32_t *cell_start, const uint32_t *pid, int32_t M,
              double dt, double lnL, const double *density, uint64_t seed, uint64_t step);
int orc_step_triplet(double *v, int64_t n, const int32_t *cell_start, const uint32_t *pid, int32_t M,
                     double dt, double lnL, const double *density, uint64_t seed, uint64_t step);
int orc_step_weighted(double *v, const double *w, int64_t n, const int32_t *cell_start,
                      const uint32_t *pid, int32_t M, double dt, double lnL, const double *density,
                      uint64_t seed, uint64_t step, int32_t mcc, double sigma0, double n_neutral,
                      double mass_ratio);

static double gauss(void)
{
    double u1 = (rand() + 1.0) / (RAND_MAX + 2.0), u2 = rand() / (RAND_MAX + 1.0);
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

#define CHECK(x)                                                    \
    do {                                                            \
        long long rc_ = (long long)(x);                             \
        if (rc_ != 0) {                                             \
            fprintf(stderr, "%s returned %lld\n", #x, rc_);         \
            return 1;                                               \
        }                                                           \
    } while (0)

int main(void)
{
    srand(7);
    const int32_t M = 9;
    const int64_t n = 700;
    double *v = malloc(sizeof(double) * 3 * n), *v0 = malloc(sizeof(double) * 3 * n);
    double *w = malloc(sizeof(double) * n), *q = malloc(sizeof(double) * 2 * n);
    double *dens = malloc(sizeof(double) * M), *mom = malloc(sizeof(double) * 14 * M);
    double *p2c = malloc(sizeof(double) * 2 * M);
    int32_t *cell = malloc(sizeof(int32_t) * n), *cs = malloc(sizeof(int32_t) * (M + 1));
    int32_t *sorted = malloc(sizeof(int32_t) * n), *partner = malloc(sizeof(int32_t) * n);
    int32_t *events = malloc(sizeof(int32_t) * M);
    uint32_t *pid = malloc(sizeof(uint32_t) * n);
    uint8_t *flag = malloc(n), *primary = malloc(n);
    for (int64_t l = 0; l < 3 * n; ++l) v[l] = gauss();
    for (int64_t l = 0; l < n; ++l) {
        cell[l] = (int32_t)(rand() % (M - 1));   /* the last cell stays empty */
        pid[l] = (uint32_t)l;
        w[l] = 0.5 + (rand() % 4);
        q[l] = 1.0;
        q[n + l] = v[l];
        primary[l] = (uint8_t)(rand() % 50 == 0);
    }
    for (int32_t j = 0; j < M; ++j) dens[j] = 0.5 + 0.1 * j;
    memcpy(v0, v, sizeof(double) * 3 * n);
    orc_params p = {0.01, 10.0, dens, 3, 4, 1, 1, 0.7, 1.0, 0.01, NULL, NULL};
    CHECK(orc_step(v, cell, pid, n, M, &p, cs));        /* bins, collides, corrects, scatters */
    p.conserve = 0;
    p.step = 5;
    CHECK(orc_step(v, cell, pid, n, M, &p, cs));
    CHECK(orc_pairs(cs, pid, M, 3, 4, sorted, partner));
    CHECK(orc_cell_moments(v, n, cs, M, mom));
    CHECK(orc_mcc(v, pid, n, 0.01, 0.7, 1.0, 0.0, 3, 6, flag));
    CHECK(orc_mcc_exact(v, pid, n, 0.01, 0.7, 1.0, 0.0, 3, 7, flag));
    CHECK(orc_p2c(q, 2, cell, n, M, p2c));
    CHECK(orc_nanbu(v, n, cs, pid, M, 0.01, 10.0, dens, 3, 8));
    CHECK(orc_step_triplet(v, n, cs, pid, M, 0.01, 10.0, dens, 3, 9));
    CHECK(orc_step_weighted(v, w, n, cs, pid, M, 0.01, 10.0, dens, 3, 10, 1, 0.7, 1.0, 0.0));
    if (orc_recombine(v, w, pid, primary, n, cs, M, 1.0, 3, 11, events) != 0) return 1;
    for (int64_t l = 0; l < 3 * n; ++l)
        if (!isfinite(v[l])) {
            fprintf(stderr, "non-finite velocity at %lld\n", (long long)l);
            return 1;
        }
    free(v); free(v0); free(w); free(q); free(dens); free(mom); free(p2c);
    free(cell); free(cs); free(sorted); free(partner); free(events); free(pid); free(flag);
    free(primary);
    puts("oracle driver ok");
    return 0;
}

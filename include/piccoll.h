/*
 * piccoll.h -- C ABI of the MI355X electron collision step.
 *
 * One time step of the electron collision operator of a PIC-DSMC solver for
 * low-temperature plasmas (Almgren-Bell, Al Awar, Geethakrishnan, Gligoric,
 * Biros, "A Portable Multi-GPU Solver for Collisional Plasmas with Coulombic
 * Interactions"):
 *   - step S1 of the PIC scheme table: electron-electron Coulomb collisions
 *     (Sec. "Coulombic Collision Kernel", Table "Coulombic Collision Steps"
 *     CCS1-CCS5, Takizuka & Abe binary collisions within a cell);
 *   - the elastic part of step S2a run by the null-collision method (Sec.
 *     "DSMC Collision Kernel", paragraph "Null Collision Method").
 *
 * Conventions shared by every entry point
 *   - All array arguments are DEVICE pointers owned by the caller; the library
 *     never frees them.  Velocities are structure-of-arrays
 *     v = [vx(0..n-1) | vy(0..n-1) | vz(0..n-1)], element type given by a
 *     pic_dtype.  Scratch memory belongs to the context and grows on demand.
 *   - Every call is asynchronous on the context's stream (given at creation).
 *     Argument errors are returned synchronously; errors found on the device
 *     (a cell id out of range) are latched and returned by pic_sync.
 *     Nothing throws across the ABI.  One context per host thread.
 *   - Code units: m_e = 1, (e^2 / 4 pi eps0)^2 = 1, per-cell electron density
 *     n_j (default 1).  Particles have uniform weights.
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11), key =
 *     (lo32(seed), hi32(seed)), counter = (c0, lo32(step), domain, c3).
 *     Domain 0, c0 = pid: word0 pairing key, word1 null-collision candidate
 *     draw, word2/word3 Coulomb uniforms.  Domain 1, c0 = pid: uniforms of a
 *     null-collision candidate.  Domain 2, c0 = cell: judge sampling.
 *     Domain 3, c3 = replica: re-pairings for labels.  Uniform mapping
 *     U(x) = ((x >> 9) + 1/2) 2^-23.  Results depend only on
 *     (seed, step, pid, cell membership), never on storage order or launch
 *     configuration, so runs are bitwise reproducible and resumable.
 */
#ifndef PICCOLL_H
#define PICCOLL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pic_ctx pic_ctx;

typedef enum {
    PIC_OK = 0,
    PIC_ERR_ARG = 1,    /* invalid argument (NULL pointer, n < 0, dt <= 0, ...) */
    PIC_ERR_RANGE = 2,  /* a cell id outside [0, n_cells) was seen on the device */
    PIC_ERR_HIP = 3,    /* a HIP runtime call failed */
    PIC_ERR_NOMEM = 4,  /* scratch memory could not be allocated */
    PIC_ERR_DTYPE = 5,  /* unknown pic_dtype */
    PIC_ERR_STATE = 6,  /* call not valid in the context's current state */
    PIC_ERR_NONFINITE = 7 /* a velocity was not finite after a step with PIC_CHECK_FINITE */
} pic_status;

typedef enum { PIC_F32 = 0, PIC_F64 = 1 } pic_dtype;

/* flags of coulomb_collide / pic_run_steps */
enum {
    PIC_CONSERVE_FIX = 1u << 0,  /* restore each cell's FP64 momentum and thermal
                                    energy after the Coulomb step; the part the
                                    output rounding leaves unmet is carried per
                                    cell into the next step (pic_conserve_reset) */
    PIC_FUSE_MCC = 1u << 1,      /* run the null-collision step (parameters from
                                    pic_set_mcc) in the same pass, after Coulomb */
    PIC_GATE = 1u << 2,          /* learned sub-cycling gate (pic_gate_*) */
    PIC_ASSUME_SORTED = 1u << 3, /* caller asserts storage is already in cell
                                    order: the re-binning kernels are not
                                    launched; the check still runs and a
                                    violation is reported as PIC_ERR_STATE */
    PIC_MOMENTS = 1u << 4,       /* write the 14 per-cell FP64 moment sums of the
                                    post-step state to the pic_set_moments_out buffer */
    PIC_CHECK_FINITE = 1u << 5   /* debug: after the step, one read of the velocities;
                                    any NaN or infinity is reported by pic_sync as
                                    PIC_ERR_NONFINITE */
};

/* Create a context on HIP device `device`, issuing work on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  *out receives the context. */
int pic_create(pic_ctx **out, int device, void *hip_stream);
/* Synchronises the stream and frees the context's scratch memory. */
void pic_destroy(pic_ctx *ctx);
/* Static string describing a pic_status. */
const char *pic_strerror(int status);
/* Waits for the context's stream, then returns (and clears) any latched
 * device error: PIC_ERR_RANGE, PIC_ERR_STATE, PIC_ERR_NONFINITE, or PIC_OK. */
int pic_sync(pic_ctx *ctx);
/* Changes the stream subsequent calls are issued on. */
int pic_set_stream(pic_ctx *ctx, void *hip_stream);
/* Caps the scratch memory the context may hold at `bytes` (0: no cap, the
 * default).  A call whose scratch would exceed it returns PIC_ERR_NOMEM before
 * anything runs and leaves its arrays unchanged. */
int pic_set_workspace_limit(pic_ctx *ctx, size_t bytes);

/* Binning, CCS1-CCS3 of the Coulombic collision steps.
 * cell_of[n] in [0, n_cells).  Writes cell_start[n_cells+1] (exclusive prefix
 * sum of the per-cell counts, cell_start[n_cells] = n) and order[n], the
 * stable counting-sort permutation: order[k] = storage index of the k-th
 * particle in cell order (ties in storage order).  Inputs are not modified.
 * n_cells <= 2^24, n <= 2^31 - 1.  Out-of-range ids: PIC_ERR_RANGE at pic_sync
 * and unspecified outputs. */
int pic_bin_cells(pic_ctx *ctx, const int32_t *cell_of, int64_t n, int32_t n_cells,
                  int32_t *cell_start, int32_t *order);

/* One Coulomb collision step, in place (Table "Coulombic Collision Steps").
 *  v        SoA velocities of `dtype`, n particles;
 *  cell_of  cell id per particle; pid  particle identity (keys the RNG);
 *  v, cell_of and pid are permuted jointly into stable cell order (callers
 *  identify particles by pid, not by storage slot; pic_unsort restores the
 *  order pid[l] = l).  Storage already in cell order is not moved.
 *  Each cell's members are ordered by (word0 of the domain-0 draw, pid);
 *  entries (2i, 2i+1) form pairs, a last odd member sits out.  Each pair
 *  (a, b) turns its relative velocity u = v_a - v_b by the Takizuka & Abe
 *  angle: tan(Theta/2) = s z with s^2 = 8 pi n_j lnLambda dt / |u|^3,
 *  z = sqrt(-2 ln U1) cos(2 pi U2), azimuth 2 pi U3 (U1, U2 from words 2, 3
 *  of a, U3 from word 2 of b); v_a += du/2, v_b -= du/2.
 *  density: n_cells per-cell densities (device, nullable => 1).
 *  step: low 32 bits enter the counter.  flags: PIC_* above.
 *  Errors: PIC_ERR_ARG (NULL arrays with n > 0, n < 0, n_cells < 1,
 *  dt <= 0, lnLambda <= 0), PIC_ERR_DTYPE, PIC_ERR_NOMEM. */
int coulomb_collide(pic_ctx *ctx, int dtype, void *v, int32_t *cell_of, uint32_t *pid,
                    int64_t n, int32_t n_cells, double dt, double lnLambda,
                    const double *density, uint64_t seed, uint64_t step, uint32_t flags);

/* Allocation-free form of coulomb_collide, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, pairs and arithmetic as
 * coulomb_collide (its kernels and results, bit for bit), restricted to
 *  - storage already in cell order (PIC_ASSUME_SORTED is implied; a violated
 *    order latches PIC_ERR_STATE at pic_sync and leaves v unchanged);
 *  - n_cells <= PIC_NOALLOC_MAX_CELLS (else PIC_ERR_RANGE, nothing runs);
 *  - cells of at most PIC_NOALLOC_MAX_CELL_F32 (binary32) or
 *    PIC_NOALLOC_MAX_CELL_F64 (binary64) members: larger cells are left
 *    unchanged and pic_sync reports PIC_ERR_STATE;
 *  - flags among PIC_FUSE_MCC, PIC_ASSUME_SORTED and PIC_MOMENTS (the buffer of
 *    pic_set_moments_out); PIC_GATE or PIC_CONSERVE_FIX give PIC_ERR_ARG.
 * Its scratch (cell starts and work lists) is a fixed device array of
 * PIC_NOALLOC_SCRATCH_BYTES per GPU, in the library's code object, whose
 * address pic_create takes once per device: the call allocates nothing.
 * Every call on a GPU shares that GPU's array, so calls that overlap on one
 * GPU (several streams or host threads) race; calls in one stream do not.
 * Other errors as coulomb_collide. */
#define PIC_NOALLOC_MAX_CELLS 65536
#define PIC_NOALLOC_MAX_CELL_F32 10240
#define PIC_NOALLOC_MAX_CELL_F64 6144
#define PIC_NOALLOC_SCRATCH_BYTES (2u << 20)
int coulomb_collide_noalloc(pic_ctx *ctx, int dtype, void *v, int32_t *cell_of, uint32_t *pid,
                            int64_t n, int32_t n_cells, double dt, double lnLambda,
                            const double *density, uint64_t seed, uint64_t step, uint32_t flags);

/* nsteps consecutive steps step0, step0+1, ... with the arguments of
 * coulomb_collide (the operator split of the PIC scheme runs several collision
 * steps between field solves, paragraph "Operator Splitting Algorithms").
 * Without PIC_ASSUME_SORTED the first step runs eagerly and re-bins unsorted
 * storage; the collision step never changes cell membership, so the other
 * steps (all nsteps with PIC_ASSUME_SORTED) are replays of one captured HIP
 * graph of a steady-state step (order check, work queue, collide pass, step
 * counter increment in device memory).  No call waits for the device: the
 * graph is captured without executing anything, kept in the context and
 * captured again when any argument, the MCC parameters, the moments buffer or
 * the scratch memory changes.  A violated order (cell ids changed between
 * replays) latches PIC_ERR_STATE and leaves v unchanged. */
int pic_run_steps(pic_ctx *ctx, int dtype, void *v, int32_t *cell_of, uint32_t *pid, int64_t n,
                  int32_t n_cells, double dt, double lnLambda, const double *density,
                  uint64_t seed, uint64_t step0, int64_t nsteps, uint32_t flags);

/* Forgets the per-cell momentum / energy shortfall carried between
 * PIC_CONSERVE_FIX steps (use when the particle set changes). */
int pic_conserve_reset(pic_ctx *ctx);

/* Parameters of the fused null-collision step (PIC_FUSE_MCC):
 * sigma(E) = sigma0 E^-1/2 with E = |v|^2/2, neutral density n_neutral,
 * electron/neutral mass ratio mass_ratio (>= 0, < 0.5), same dt as Coulomb. */
int pic_set_mcc(pic_ctx *ctx, double sigma0, double n_neutral, double mass_ratio);

/* Stand-alone null-collision Monte Carlo step, in place (paragraph "Null
 * Collision Method"; collision probability 1 - exp(-dt |v| sigma n_n) of the
 * DSMC collision step).  For sigma = sigma0 E^-1/2 the frequency
 * nu = n_n sigma0 sqrt(2) does not depend on speed, so nu_max = nu and every
 * candidate is real.  A particle is a candidate iff word1 of its domain-0
 * draw < floor(P_null 2^32), P_null = 1 - exp(-nu_max dt); candidates scatter
 * elastically and isotropically (domain 1: cos theta = 1 - 2 U(w1),
 * phi = 2 pi U(w2)) with |v'|^2 = |v|^2 (1 - 2 mass_ratio (1 - vhat.s)).
 * Storage order is irrelevant and unchanged.  candidate_out (nullable,
 * uint8[n]) receives the candidate flags. */
int mcc_null_collide(pic_ctx *ctx, int dtype, void *v, const uint32_t *pid, int64_t n,
                     double dt, double sigma0, double n_neutral, double mass_ratio,
                     uint64_t seed, uint64_t step, uint8_t *candidate_out);

/* ---------------------------------------------------------------- DSMC-Coll */
/* Electron-heavy collisions of the paper's collision table, C1 elastic, C2
 * ionization and C3 metastable excitation on the ground-state density, C4
 * two-step ionization on the metastable density (Table "DSMC Collision Step",
 * CS0-CS5, and the probability pi_c = 1 - exp(-dt |v| sigma_c(E) n_k) of
 * the section "DSMC Collision Kernel").  Cross sections (host arrays,
 * copied): piecewise cubic in E = |v|^2 / 2 on breakpoints breaks[0] = 0 <
 * ... < breaks[nseg] (1 <= nseg <= 64), coef[(c * nseg + p) * 4 + q] the
 * coefficient of (E - breaks[p])^q on segment p of channel c (0..3); constant
 * beyond breaks[nseg], clipped at 0, zero below threshold[c] (the channel's
 * energy loss; threshold[0] is normally 0).  mass_ratio: elastic speed loss.
 * PIC_ERR_ARG on bad input. */
int pic_set_dsmc(pic_ctx *ctx, int32_t nseg, const double *breaks, const double *coef,
                 const double *threshold, double mass_ratio);
/* One DSMC-Coll step of the n particles (v SoA stride n, any storage
 * order): per particle one domain-6 draw; U(word 0) picks the first channel
 * whose cumulative probability exceeds it (none: no collision); the scattered
 * direction is cos = 1 - 2 U(word 1), phi = 2 pi U(word 2); elastic keeps |v|
 * up to the m/M loss; excitation loses threshold[2]; ionization loses its
 * threshold and splits the rest U(word 3) : 1 - U(word 3) with a new
 * electron whose direction uses words 1, 2 of the domain-7 draw.  The new
 * electron is appended at slot *count (device uint64, read and advanced
 * atomically, so the order of new electrons is arbitrary) of v_new (SoA stride
 * cap), pid_new = pid_base + parent pid, cell_new = parent cell; beyond cap it
 * is counted but not written and pic_sync reports PIC_ERR_STATE.  Densities:
 * n_gas / n_meta device per-cell arrays [n_cells] indexed by cell_of, or the
 * scalars when NULL; a particle whose cell is outside [0, n_cells) is left
 * alone and pic_sync reports PIC_ERR_RANGE.  channel_out (nullable,
 * uint8[n]): 0 none, 1..4 = C1..C4. */
int dsmc_collide(pic_ctx *ctx, int dtype, void *v, const int32_t *cell_of, const uint32_t *pid,
                 int64_t n, int32_t n_cells, const double *n_gas, const double *n_meta, double n_gas0,
                 double n_meta0, double dt, uint64_t seed, uint64_t step, uint32_t pid_base,
                 void *v_new, uint32_t *pid_new, int32_t *cell_new, int64_t cap, uint64_t *count,
                 uint8_t *channel_out);

/* Exact-count variant of the null-collision step (the paper selects P_null N
 * particles at random, paragraph "Null Collision Method"): exactly
 * K = round(P_null n) particles scatter, those with the K smallest candidate
 * words (word 1 of the domain-0 draw, the word the per-particle test of
 * mcc_null_collide compares with floor(P_null 2^32)), equal words ordered by
 * (pid, slot) -- a uniformly random K-subset, and the particles the
 * per-particle test picks are a subset or a superset of it.  Scattering as in
 * mcc_null_collide.  pid holds particle ids (unique in normal use; particles
 * sharing the threshold word are ranked pairwise, at a cost quadratic in
 * their number).  Uses context scratch (8 bytes per particle, 8 per
 * selected one).
 * selected_out (nullable, n bytes) receives 1 for a selected particle.
 * Errors: PIC_ERR_ARG (n < 0 or n > 2^31 - 1, NULL arrays with n > 0,
 * dt <= 0, negative sigma0, n_neutral or mass ratio, mass ratio >= 1/2),
 * PIC_ERR_DTYPE, PIC_ERR_NOMEM. */
int mcc_null_collide_exact(pic_ctx *ctx, int dtype, void *v, const uint32_t *pid, int64_t n,
                           double dt, double sigma0, double n_neutral, double mass_ratio,
                           uint64_t seed, uint64_t step, uint8_t *selected_out);

/* Nanbu's Coulomb operator (the alternative to the Takizuka & Abe method the
 * paper names in its related work) on the pairs of coulomb_collide: same
 * pairing (the cell's members ordered by (word 0, pid) of the step's draw,
 * pairs (2i, 2i+1)); the pair (a, b), a the lower slot, turns its relative
 * velocity u by chi with cos chi distributed as exp(A cos chi), A solving
 * coth A - 1/A = exp(-s), s = 16 pi n lnLambda dt / |u|^3 (twice the Takizuka
 * & Abe variance of tan(Theta/2), so both have the same small-angle
 * diffusion); U = U(word 2 of a) inverts its distribution function, the
 * azimuth is 2 pi U(word 2 of b).  Momentum and energy of each pair are kept.
 * Storage in cell order, cell_start of n_cells + 1 entries; density per cell
 * (nullable: 1).  Arithmetic in binary64 for either dtype.  Errors:
 * PIC_ERR_ARG (NULL arrays with n > 0, n < 0 or n > 2^31 - 1, n_cells < 1,
 * dt <= 0, lnLambda <= 0), PIC_ERR_DTYPE, PIC_ERR_NOMEM. */
int coulomb_collide_nanbu(pic_ctx *ctx, int dtype, void *v, const uint32_t *pid, int64_t n,
                          const int32_t *cell_start, int32_t n_cells, double dt, double lnLambda,
                          const double *density, uint64_t seed, uint64_t step);

/* The Takizuka & Abe step with their triplet for odd cells (the paper's
 * odd-cell handling, paragraph on the Coulomb kernel, leaves the last member
 * idle): same pairing and pair arithmetic as coulomb_collide (no null
 * collisions, no correction); in a cell of odd N >= 3 the last three members
 * in pairing order, p0 p1 p2, collide pairwise at dt/2 in the order
 * (p0, p1), (p1, p2), (p2, p0), each on the velocities the previous one left,
 * with the uniforms of Philox domains 0, 4 and 5 respectively.  Cells of
 * even size give exactly coulomb_collide's velocities.  Storage in cell
 * order, cell_start of n_cells + 1 entries; density per cell (nullable: 1).
 * Errors as coulomb_collide_nanbu. */
int coulomb_collide_triplet(pic_ctx *ctx, int dtype, void *v, const uint32_t *pid, int64_t n,
                            const int32_t *cell_start, int32_t n_cells, double dt, double lnLambda,
                            const double *density, uint64_t seed, uint64_t step);

/* The Takizuka & Abe step for particles of unequal weight (the paper uses
 * uniform weights and names weights that differ between particles as the
 * next step, Sec. "Conclusion").  Rule (Nanbu & Yonemura's for weighted
 * binary collisions): the pairs and each pair's half change h are
 * coulomb_collide's; the member of smaller weight w_l always takes its half
 * change, the other one iff U4 * w_h < w_l in binary64, with U4 the uniform
 * of word 3 of the second member's domain-0 draw.  Equal weights give
 * coulomb_collide's velocities; weighted momentum and energy are conserved
 * on average.  w: n weights (>= 0) of `dtype`, not modified.  Storage in cell
 * order (v, w and pid), cell_start of n_cells + 1 entries; density per cell
 * (nullable: 1).  flags: 0 or PIC_FUSE_MCC (null collisions as
 * coulomb_collide's, PIC_ERR_STATE before pic_set_mcc).  Errors as
 * coulomb_collide_nanbu, PIC_ERR_ARG for a NULL w or other flags. */
int coulomb_collide_weighted(pic_ctx *ctx, int dtype, void *v, const void *w, const uint32_t *pid,
                             int64_t n, const int32_t *cell_start, int32_t n_cells, double dt,
                             double lnLambda, const double *density, uint64_t seed, uint64_t step,
                             uint32_t flags);

/* Recombination C5 (section "Kernel for Recombination Collision C5", table
 * "Recombination Steps" RS1-RS5): in each cell the live primaries
 * (primary[l] != 0, w[l] > 0; the paper's list from step CS3) are matched one
 * to one with the live catalytes (primary[l] == 0, w[l] > 0) of the same
 * cell.  The paper pops catalytes from per-cell lists with atomics; here the
 * matching is fixed: the k-th primary in storage order takes the catalyte of
 * rank (o_j + k) mod C_j in storage order, o_j = floor(word0 C_j / 2^32) of a
 * Philox draw (domain 9, counter = cell index), for k < min(P_j, C_j).  The
 * catalyte's speed becomes sqrt(2 (|v_c|^2/2 + |v_p|^2/2 + eps)) in an
 * isotropic direction (words 1, 2 of a domain-8 draw on its pid); the
 * primary's weight becomes 0 (RS5).  Storage in cell order: cell_start of
 * n_cells + 1 entries as pic_bin_cells returns.  v (3 x n SoA) and w (n)
 * of the velocity dtype, updated in place; events (nullable, n_cells int32)
 * receives min(P_j, C_j).  Errors: PIC_ERR_ARG (NULL arrays with n > 0,
 * n < 0 or n > 2^31 - 1, n_cells < 1, eps negative or not finite),
 * PIC_ERR_DTYPE. */
int recombine(pic_ctx *ctx, int dtype, void *v, void *w, const uint32_t *pid, const uint8_t *primary,
              int64_t n, const int32_t *cell_start, int32_t n_cells, double eps, uint64_t seed,
              uint64_t step, int32_t *events);

/* Particle-to-cell sums (section "Particle-to-Cell"; steps S3a-S3b of the
 * PIC scheme table): out[j * nq + k] = sum over the particles l with
 * cell_of[l] == j of q[k * n + l], for cells j < n_cells and quantities
 * k < nq.  q: nq rows of n values (SoA), binary32 or binary64 by dtype;
 * particles in any order; sums accumulated in binary64, so the result can
 * differ from one call to the next in the last bits (the order of the
 * atomic additions is not fixed).  out: n_cells * nq doubles, overwritten.
 * A cell id outside [0, n_cells) is skipped and pic_sync reports
 * PIC_ERR_RANGE.  Errors: PIC_ERR_ARG (NULL arrays with n > 0, n < 0 or
 * n > 2^31 - 1, n_cells < 1, nq outside 1..4, n_cells * nq > 2^28),
 * PIC_ERR_DTYPE, PIC_ERR_NOMEM (scratch of up to 8 copies of out). */
int p2c_sums(pic_ctx *ctx, int dtype, const void *q, int32_t nq, const int32_t *cell_of, int64_t n,
             int32_t n_cells, double *out);

/* Device buffer of n_cells * 14 doubles receiving the post-step moment sums
 * (layout of pic_cell_moments) when PIC_MOMENTS is passed; NULL clears it. */
int pic_set_moments_out(pic_ctx *ctx, double *out);

/* ---------------------------------------------------------------- learned gate */
/* A per-cell network decides which cells may defer their Coulomb collision
 * (sub-cycling): a deferred cell keeps its velocities apart from null
 * collisions, counts k, and later collides once with dt_eff = (k + 1) dt.
 * Not part of the paper; its method is the plain operator, which stays the
 * fallback and the judge. */

#define PIC_MLP_PARAMS 4801
/* Parameter layout (binary32): W1[8][64] at 0, b1[64] at 512, W2[64][64] at
 * 576, b2[64] at 4672, W3[64] at 4736, b3 at 4800; logit =
 * W3 . relu(W2^T relu(W1^T x + b1) + b2) + b3, probability = logistic(logit).
 * bf16 != 0: products of bfloat16-rounded weights, inputs and activations
 * with binary32 accumulation. */

/* Features from per-cell raw sums (layout of pic_cell_moments), feat[8*j..]:
 * ln N, ln T, T_xx/T - 1, T_yy/T - 1, T_zz/T - 1, ||offdiag T||_F/T, |q|/(N T^1.5),
 * <|c|^4>/(15 T^2) - 1 with c = v - V, T_ab = <c_a c_b>, T = tr/3,
 * q = 1/2 sum |c|^2 c.  Cells with N < 2 or T <= 0: zeros, valid[j] = 0
 * (valid nullable). */
int pic_features(pic_ctx *ctx, const double *moments, int32_t n_cells, float *feat, uint8_t *valid);

/* Expected relative one-step relaxation of each cell's temperature tensor
 * (storage in cell order): r_j = ||(1/K) sum over K re-pairings (domain 3,
 * c3 = replica) of sum_pairs 1/4 h(s^2) (|u|^2 I - 3 u u^T)||_F / (N_j T_j),
 * h(s^2) = E[sin^2 Theta] of the Takizuka & Abe angle, s^2 from dt times
 * dt_scale[j] (nullable => 1).  Cells with fewer than 2 members: 0. */
int pic_relaxation(pic_ctx *ctx, int dtype, const void *v, int64_t n, const int32_t *cell_start,
                   const uint32_t *pid, int32_t n_cells, double dt, double lnLambda,
                   const double *density, const double *dt_scale, uint64_t seed, uint64_t step,
                   int32_t replicas, double *r_out);

/* Estimate of pic_relaxation's r_j from the moment sums alone (layout of
 * pic_cell_moments; no pairing), the baseline gate the network is compared
 * with: r^2 = r_aniso^2 + r_floor^2, r_aniso = 3 nu_0 dt ||A||_F for the
 * traceless part A of the temperature tensor in units of T (linearised
 * isotropisation, nu_0 = (8 sqrt(pi) / 15) n lnL / T^1.5), and
 * r_floor^2 = (8 pi n lnL dt / T^1.5)^2 / N (a - b + (3/2 - a) / K), the
 * small-angle spread of the pair sum of an isotropic Maxwellian cell over
 * random pairings, a = 6 E[psi^2] = 0.1521598 (psi from the Maxwellian's
 * Rosenbluth potential), b = 10 / (25 pi), K = replicas.  density per cell
 * (device, nullable: 1).  r_out: device double[n_cells]; NaN for cells of
 * fewer than 2 members or no temperature.  PIC_ERR_ARG for NULL arrays,
 * n_cells < 1, dt <= 0, lnLambda <= 0 or replicas < 1. */
int pic_analytic_relaxation(pic_ctx *ctx, const double *moments, int32_t n_cells, double dt,
                            double lnLambda, const double *density, int32_t replicas, double *r_out);

/* prob[b] = network output for x[8*b .. 8*b+7]. */
int pic_mlp_forward(pic_ctx *ctx, const float *params, const float *x, int32_t batch, int bf16,
                    float *prob);
/* Gradient of the mean binary cross-entropy of the logits against y[batch]
 * (0/1) with respect to the 4801 parameters; loss (device, nullable) gets the
 * mean loss.  Summation order is fixed (bitwise reproducible). */
int pic_mlp_grad(pic_ctx *ctx, const float *params, const float *x, const float *y, int32_t batch,
                 int bf16, float *grad, float *loss);
/* pic_mlp_grad followed by one Adam step (beta1 0.9, beta2 0.999, eps 1e-8,
 * bias-corrected with step t >= 1) on the binary32 master parameters. */
int pic_mlp_train_step(pic_ctx *ctx, float *params, float *adam_m, float *adam_v, int32_t t,
                       float lr, const float *x, const float *y, int32_t batch, int bf16,
                       float *loss);
/* One bfloat16 training step in the boundary's short form: feat float[8
 * batch] (layout of pic_features), label float[batch] (1: r < tolerance),
 * w_master float[4801] (binary32 master parameters, updated in place),
 * adam_state float[2 * 4801] (first moments, then second moments; zero before
 * the first step), loss_out (device, nullable) the batch's mean loss.  The
 * Adam step count is kept by the context: it restarts at 1 whenever w_master
 * differs from the previous call's and counts up otherwise.  Same arithmetic
 * as pic_mlp_train_step with bf16 = 1. */
int mlp_train_step(pic_ctx *ctx, const void *feat, const float *label, int32_t batch, void *w_master,
                   void *adam_state, float lr, float *loss_out);

/* Stand-alone gate decision for features feat[8 n_cells] (layout of
 * pic_features): prob = the network (bf16 as in pic_mlp_forward), then
 * skip[j] = prob > threshold and k_acc[j] < k_max; k_acc[j] (deferred-step
 * count, device, read and updated) becomes k_acc[j] + 1 for a skipped cell and
 * 0 otherwise.  prob_out (device float[n_cells], nullable) receives the
 * probabilities.  No judge and no dt scale: that is the PIC_GATE step. */
int gate_infer(pic_ctx *ctx, const float *feat, int32_t n_cells, const float *params, float threshold,
               int32_t k_max, int bf16, uint8_t *skip, int32_t *k_acc, float *prob_out);

/* Enables PIC_GATE steps: params (device, kept by pointer), skip when the
 * probability exceeds threshold and the cell has deferred fewer than k_max
 * steps; on the steps that refresh the moment sums (pic_gate_refresh) a
 * judge_fraction of cells (domain-2 draw per cell and step) always collides
 * and is scored: a judged cell the network wanted to skip is a false skip if
 * its relaxation (replicas re-pairings) reaches tolerance.  When more than 10%
 * of at least 20 judged skips are false the gate switches itself off (all
 * cells collide).  The first gated step collides every cell and records the
 * moments the next step decides from.  Deferred cells enter no collision
 * queue; with PIC_FUSE_MCC their null collisions still run.  With
 * PIC_MOMENTS the moment sums of every cell are written after the step. */
int pic_gate_config(pic_ctx *ctx, const float *params, float threshold, int32_t k_max,
                    double judge_fraction, double tolerance, int32_t replicas, int bf16);
/* The same gate with the analytic estimate of pic_analytic_relaxation in
 * place of the network: a cell may skip when its estimate over the
 * tolerance is below threshold (from the gate's refreshed moments, with the
 * step's dt, lnLambda and densities and K = replicas).  Judge, switch-off,
 * refresh and deferral as pic_gate_config, which it replaces (as that
 * replaces it).  pic_gate_state's prob receives estimate / tolerance. */
int pic_gate_config_analytic(pic_ctx *ctx, float threshold, int32_t k_max, double judge_fraction,
                             double tolerance, int32_t replicas);
/* Moment refresh interval of the gate: the 14 moment sums its features come
 * from are recomputed (a streaming pass over the post-step velocities) on
 * the first gated step and then on steps that are multiples of `every`
 * (default 1: every step); in between the network reads the last refresh and
 * no cell is judged.  The choice is made on the device, so graph replays
 * follow it.  PIC_ERR_ARG if every < 1. */
int pic_gate_refresh(pic_ctx *ctx, int32_t every);
/* Forgets deferred counts, moments and statistics. */
int pic_gate_reset(pic_ctx *ctx);
/* Host int64 out[8]: gated steps, cells skipped, cells collided, cells
 * judged, judged cells the network wanted to skip, false skips, switched off,
 * moments present.  Synchronises. */
int pic_gate_stats(pic_ctx *ctx, int64_t *out);
/* Device copies of the last gate decisions (each nullable): skip[n_cells],
 * k_acc[n_cells], prob[n_cells], moments[14 n_cells]. */
int pic_gate_state(pic_ctx *ctx, uint8_t *skip, int32_t *k_acc, float *prob, double *moments);

/* Batching.  Cells go to size classes (workgroup-per-cell kernels of 256,
 * 512 and 1024 threads holding up to 512 / 2048 / 4096 / 10240 members in
 * binary32, 256 / 2048 / 4096 / 6144 in binary64, and a multi-block class
 * beyond), each a persistent kernel draining its work list.  The plain step
 * (with or without PIC_FUSE_MCC) can instead run its whole collide pass as
 * one persistent launch (the paper runs several steps per kernel call to
 * avoid relaunch costs, paragraph "Operator Splitting Algorithms"): the
 * segments of the largest cells first, then the other cells largest first on
 * whole workgroups, and when that queue is empty every wave takes cells of
 * the smallest class one at a time (or every cell on whole workgroups).
 * pic_set_schedule picks the form for a dtype: 0 one launch per class (the
 * default), 1 one launch with the wave schedule for the smallest class, 2 one
 * launch with every cell on whole workgroups; it keeps the class thresholds
 * and replaces an earlier pic_autotune choice.  Results do not depend on the
 * form, bit for bit.  PIC_ERR_ARG for another schedule.  pic_autotune
 * times candidate routing thresholds and resident-workgroup counts for the
 * given state on a scratch copy (the caller's arrays are not modified; it
 * synchronises and allocates) and keeps the fastest for later steps of this
 * dtype on the context.  If the environment variable PICCOLL_TUNE_CACHE
 * names a file, choices are read from and appended to it as JSON lines keyed
 * by (device architecture, dtype, n, n_cells, flags, histogram of log2 cell
 * sizes).  *choice_out (nullable) receives the chosen candidate index.
 * Flags PIC_GATE, PIC_MOMENTS and PIC_ASSUME_SORTED are ignored here. */
int pic_set_schedule(pic_ctx *ctx, int dtype, int schedule);
int pic_autotune(pic_ctx *ctx, int dtype, const void *v, const int32_t *cell_of,
                 const uint32_t *pid, int64_t n, int32_t n_cells, double dt, double lnLambda,
                 uint32_t flags, int32_t *choice_out);

/* ---------------------------------------------------------------- measurement */

/* on != 0: record HIP events around the library's kernel launches on the
 * context's stream (for benchmarks; adds two event records per launch). */
int pic_time_kernels(pic_ctx *ctx, int on);
/* Waits for the recorded events and returns, per slot, the summed elapsed
 * milliseconds ms[16] and launch counts count[16] since the previous call,
 * then forgets them.  Slots: 0-3 collide pass of the LDS size classes
 * (cells of at most 512 / 2048 / 4096 / 10240 members in binary32,
 * 512 / 2048 / 4096 / 6144 in binary64), 4 cells beyond those, 5 order check
 * and cell starts, 6 work queue, 7 re-binning passes, 8 stand-alone
 * null-collision step, 9 learned-gate decision, 10 relaxation of the
 * judged cells, 11 null collisions of deferred cells, 12 gate's moment
 * pass, 13 DSMC-Coll step, 14 particle-to-cell sums, 15 recombination, 16
 * Nanbu step (pairing and rotation), 17 triplet step (pairing and collisions)
 * (ms and count hold 20 slots). */
int pic_kernel_times(pic_ctx *ctx, double *ms, int64_t *count);

/* ---------------------------------------------------------------- test exports */

/* out[4*i + w] = word w of Philox4x32-10 with counter (c0[i], lo32(step),
 * domain, c3) and key (lo32(seed), hi32(seed)). */
int pic_philox(pic_ctx *ctx, uint64_t seed, uint64_t step, uint32_t domain, uint32_t c3,
               const uint32_t *c0, int64_t n, uint32_t *out);

/* The pairing of the Coulomb step (partner pairs within each cell's list,
 * steps CCS3-CCS5 of Table "Coulombic Collision Steps"; the order inside a
 * cell is random: sorted by (word 0 of the member's domain-0 draw, pid), pairs
 * (0,1), (2,3), ...; an odd cell's last member is idle) for storage already
 * in cell order (cell_start from pic_bin_cells):
 * sorted[cell_start[j] + r] = slot of the r-th member of cell j in
 * (key, pid) order; partner[slot] = partner slot or -1 (idle).  Device
 * arrays of n (= cell_start[n_cells]) entries.  PIC_ERR_ARG for NULL arrays
 * or n_cells < 1. */
int coulomb_pairs(pic_ctx *ctx, const int32_t *cell_start, const uint32_t *pid,
                  int32_t n_cells, uint64_t seed, uint64_t step, int32_t *sorted,
                  int32_t *partner);

/* Per-cell FP64 raw moment sums of storage in cell order, out[14*j + k]:
 * N, sum vx, vy, vz, sum vx^2, vy^2, vz^2, sum vx vy, vx vz, vy vz,
 * sum |v|^2 vx, |v|^2 vy, |v|^2 vz, sum |v|^4.  The first seven carry each
 * cell's momentum and energy, which every partner pair of step CCS5 (Table
 * "Coulombic Collision Steps") conserves; the rest feed the gate's features.
 * out: device double[14 n_cells].  PIC_ERR_ARG for NULL arrays or
 * n_cells < 1. */
int pic_cell_moments(pic_ctx *ctx, int dtype, const void *v, int64_t n,
                     const int32_t *cell_start, int32_t n_cells, double *out);

/* Undoes the re-binning (step CCS3 of Table "Coulombic Collision Steps"
 * moves particles into cell order here, where the paper sorts indices):
 * restores storage to pid order (slot pid[k] receives particle k), i.e. the
 * caller's original order when pid was 0..n-1.  pid must be a permutation of
 * 0..n-1 (not checked). */
int pic_unsort(pic_ctx *ctx, int dtype, void *v, uint32_t *pid, int32_t *cell_of, int64_t n);

#ifdef __cplusplus
}
#endif
#endif /* PICCOLL_H */

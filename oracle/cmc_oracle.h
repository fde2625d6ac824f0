/*
 * cmc_oracle.h -- plain, serial, FP64 CPU oracle of one Henon Monte Carlo step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no source
 * with the HIP library and must never be called from the product path.
 *
 * Method: Pattabiraman et al., "A Parallel Monte Carlo Code for Simulating
 * Collisional N-body Systems" (arXiv:1206.5878), Sec. 2.1 (the serial step:
 * potential, timestep, two-body relaxation, new orbits, sort) and Sec. 3.2
 * (20-star radial bins).  Units: G = 1, total mass 1 (Henon units).
 * Stars are 0-based here; the paper counts from 1.
 *
 * Every function is written for clarity, not speed: straight loops, Neumaier
 * compensated sums, bisection searches, qsort.  Random numbers come from
 * Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11) keyed by the run seed with
 * counter (star id, step, purpose, trial); see the purpose codes below.
 */
#ifndef CMC_ORACLE_H
#define CMC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Philox counter word 2: what the draw is for. */
enum {
  ORA_P_INIT_POS = 0x10,   /* radius uniform X1 and direction uniform X6       */
  ORA_P_INIT_SPEED = 0x11, /* speed rejection trial j: (q, X5)                 */
  ORA_P_INIT_MASS = 0x12,  /* mass-spectrum segment and inverse-CDF uniforms   */
  ORA_P_RELAX = 0x20,      /* pair azimuths psi and psi'                       */
  ORA_P_ORBIT = 0x30,      /* rejection trial j: (X, X')                       */
  ORA_P_SIGN = 0x31,       /* sign of the new radial velocity                  */
  ORA_P_ENSEMBLE = 0x40    /* ensemble cluster sizes                           */
};

/* Status bits (sticky, OR-ed together). */
enum {
  ORA_ST_NONFINITE = 1u << 0,  /* a non-finite value appeared                  */
  ORA_ST_TRIAL_CAP = 1u << 1,  /* rejection sampling hit the trial cap         */
  ORA_ST_BOUND = 1u << 2,      /* the sampling bound F was exceeded            */
  ORA_ST_ESCAPER = 1u << 3,    /* at least one star had E >= 0                 */
  ORA_ST_DT_DEGEN = 1u << 4,   /* no positive dt reaches the target            */
  ORA_ST_NUMERIC = 1u << 5     /* degenerate orbit (infinite sampling bound)   */
};

/* ---- random numbers ---------------------------------------------------- */
void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void ora_philox_many(int64_t n, uint64_t key, const uint32_t *ctr, uint32_t *out);
double ora_u01(uint32_t hi, uint32_t lo); /* (2x+1) 2^-53, x = top 52 bits   */
float ora_u01f(uint32_t hi);              /* (2x+1) 2^-24, x = top 23 bits   */

/* The generator of Sec. 3.6: L'Ecuyer's combined Tausworthe LFSR113 (four
 * component LFSRs, degrees 31, 29, 28, 25; state z[0..3], component c keeps
 * the top k_c bits of z[c]; a usable state has each of those parts nonzero).
 * next: one 32-bit output; block: 4 consecutive outputs (one draw of the
 * step, in place of one Philox block). */
uint32_t ora_lfsr113_next(uint32_t z[4]);
void ora_lfsr113_block(uint32_t z[4], uint32_t w[4]);
/* z advanced by 2^e steps (the e-fold squared step matrix of each component). */
void ora_lfsr113_jump_pow2(uint32_t z[4], int e);
/* Stream `id` of the seed state z0: z0 advanced by id * 2^80 steps, the jump
 * displacement of Sec. 3.6. */
void ora_lfsr113_stream(const uint32_t z0[4], uint64_t id, uint32_t z[4]);
/* Pin helper: steps until component c's state (its top k bits) returns to
 * that of z, or -1 after `limit` steps. */
int64_t ora_lfsr113_component_period(int c, uint32_t z, int64_t limit);

/* ---- initial model (Sec. 2.1 opening paragraph) ------------------------- */
/* Plummer model, unsorted, star i gets id i.  mass_spectrum: 0 = equal
 * masses 1/n, 1 = broken power law (slope -1.3 on [0.1,0.5], -2.3 on
 * [0.5,100]) rescaled to total mass 1. */
void ora_plummer(int64_t n, uint64_t seed, int mass_spectrum, double *r, double *vr,
                 double *vt, double *m, uint32_t *id);

/* King density rho(W) up to a constant: e^W erf(sqrt W) - sqrt(4W/pi)(1 + 2W/3). */
double ora_king_density(double W);

/* King (1966) profile for central potential w0: nodes (r, W, M) into
 * rk/Wk/Mk (at most cap), tail = (r_t, M_t, W_pot); returns the node count. */
int ora_king_profile(double w0, double *rk, double *Wk, double *Mk, int cap, double *tail);

/* n stars of a King model, unsorted, in Henon units (see cmc_oracle.c). */
void ora_king(int64_t n, uint64_t seed, double w0, int mass_spectrum, double *r, double *vr,
              double *vt, double *m, uint32_t *id);

/* ---- step 6 of Sec. 2.1: sort ------------------------------------------- */
/* perm[p] = old index of the star that lands at position p, ascending in the
 * key, equal keys in old-index order (a stable sort). */
void ora_sort_perm(int64_t n, const double *key, int64_t *perm);

/* ---- step 1 of Sec. 2.1: potential ---------------------------------------- */
/* phi[k] = -(mcum[k]/r[k] + ssuf[k]); mcum = inclusive mass prefix, ssuf =
 * exclusive suffix of m/r (may be NULL). */
void ora_potential(int64_t n, const double *r, const double *m, double *phi, double *mcum,
                   double *ssuf);

/* ---- step 2 (replaced) and 3 of Sec. 2.1 + Sec. 3.2 bins ------------------ */
/* Per pair p = (2p, 2p+1): relative speed w and representative-encounter
 * time t_p (t_p = +inf for a massless pair, 0 for a zero-volume bin). Returns
 * the number of pairs, floor(n/2). */
int64_t ora_pair_terms(int64_t n, const double *r, const double *m, const double *vr,
                       const double *vt, const uint32_t *id, uint64_t seed, uint32_t step,
                       double gamma, double *w, double *tp, double *nb);
/* Mean of sin^2(beta_p/2) over pairs with w > 0 for a given dt. */
double ora_mean_sin2(int64_t np, const double *w, const double *tp, double dt);
/* dt with mean sin^2(beta/2) = target; *status gets ORA_ST_DT_DEGEN when none. */
double ora_solve_dt(int64_t np, const double *w, const double *tp, double target,
                    uint32_t *status);

/* Pair kicks in place (vr, vt) for a given dt. */
void ora_relax(int64_t n, const double *r, const double *m, double *vr, double *vt,
               const uint32_t *id, uint64_t seed, uint32_t step, double gamma, double dt);

/* ---- step 5 of Sec. 2.1: new orbits --------------------------------------- */
typedef struct {
  int64_t n_esc;       /* stars with E >= 0                                    */
  int64_t trials;      /* total rejection trials                               */
  int64_t violations;  /* trials with g(s0) > F                                */
  int64_t capped;      /* stars that hit the trial cap                         */
  double e_esc;        /* sum m E over escapers                                */
  uint32_t status;
} ora_orbit_stats;

/* For every star: E, J, bracket intervals, roots, rejection sample.  Writes
 * r_new (+inf for escapers) and overwrites vr, vt with the new velocities.
 * Optional per-star outputs may be NULL; flags_out holds the status bits
 * raised by that star. */
void ora_orbit(int64_t n, const double *r, const double *phi, const double *mcum,
               const double *ssuf, const double *m, double *vr, double *vt, const uint32_t *id, uint64_t seed,
               uint32_t step, int32_t trial_cap, double bound_factor, double *r_new,
               double *E_out, double *J_out, int64_t *kmin_out, int64_t *kmax_out,
               double *rmin_out, double *rmax_out, int32_t *trials_out,
               uint32_t *flags_out, ora_orbit_stats *st);

/* ora_orbit for the listed stars only (idx[0..count-1]): writes r_new, vr,
 * vt at those indices; every other entry is left alone.  Each star's new
 * orbit depends on the table and its own state only, so this is ora_orbit
 * restricted to a sample (for checks at sizes where the whole pass is slow). */
void ora_orbit_subset(int64_t n, const double *r, const double *phi, const double *mcum,
                      const double *ssuf, const double *m, double *vr, double *vt,
                      const uint32_t *id, uint64_t seed, uint32_t step, int32_t trial_cap,
                      double bound_factor, int64_t count, const int64_t *idx, double *r_new);

/* Potential at an arbitrary radius from the table. */
double ora_phi_at(int64_t n, const double *r, const double *phi, const double *mcum,
                  const double *ssuf, double x);

/* ---- one whole step --------------------------------------------------------- */
typedef struct {
  uint64_t seed;
  uint32_t step;
  double gamma;        /* Coulomb logarithm ln(gamma N)                        */
  double target;       /* mean sin^2(beta/2) that fixes dt                     */
  double dt_fixed;     /* > 0: use this dt instead of solving                  */
  int32_t trial_cap;
  double bound_factor;
} ora_params;

typedef struct {
  double dt;
  int64_t n_after;
  ora_orbit_stats orbit;
  uint32_t status;
} ora_step_out;

/* potential -> pair terms -> dt -> relax -> orbit -> sort, in place on the
 * SoA arrays (length n on entry, n_after on exit).  phi/mcum receive the table
 * of the state at entry. */
void ora_step(int64_t n, double *r, double *vr, double *vt, double *m, uint32_t *id,
              double *phi, double *mcum, const ora_params *p, ora_step_out *out);

/* ora_step that also reports, for the star at each position q < n_after of
 * the new state, moves[3q..3q+2] = (r_old, Phi_old(r_old), Phi_old(r_new)):
 * its radius before the step and the old potential there and at its new
 * radius.  moves may be NULL.  lfsr (4 words per star, or NULL for Philox):
 * every draw of the step is the next block of the drawing star's own LFSR113
 * stream -- the pair's first star for a relaxation, the star itself for each
 * rejection trial and then its sign -- and the states move with the stars. */
void ora_step_ex(int64_t n, double *r, double *vr, double *vt, double *m, uint32_t *id,
                 double *phi, double *mcum, const ora_params *p, ora_step_out *out,
                 double *moves, uint32_t *lfsr);

/* ---- energy correction (Sec. 2.1 item 6) ----------------------------------- */
/* For the state a step produced (n stars, its potential phi) and that step's
 * moves: dT = (dPhi(r_old) - dPhi(r_new)) / 2 per unit mass with
 * dPhi = Phi_new - Phi_old, Phi_new(r_old) from the defining sum over the n
 * stars; vr, vt scaled by sqrt(1 + 2 dT / v^2) in place.  Returns the number
 * of stars left unchanged because v^2 + 2 dT <= 0 or v = 0 (with dT != 0). */
int64_t ora_energy_correction(int64_t n, const double *r, const double *m, double *vr,
                              double *vt, const double *phi, const double *moves);

/* ---- diagnostics ------------------------------------------------------------ */
/* out[0]=T, out[1]=W, out[2]=E=T+W, out[3]=2T/|W|, out[4]=M, out[5..8]=
 * Lagrange radii for 1%, 10%, 50%, 90% of the mass, out[9] = density-weighted
 * core radius r_c, out[10] = core density rho_c (NaN when n < 7).  Needs
 * phi/mcum of the same state. */
void ora_diagnostics(int64_t n, const double *r, const double *vr, const double *vt,
                     const double *m, const double *phi, const double *mcum, double *out);

/* Threads the parallel loops use: 1 for the plain build, the OpenMP team
 * size for the OpenMP build (liboracle_omp.so). */
int ora_threads(void);

#ifdef __cplusplus
}
#endif
#endif

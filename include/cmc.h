/*
 * cmc.h -- C ABI of libcmc.so: one Henon Monte Carlo step of a spherical star
 * cluster on an AMD Instinct MI355X (gfx950), written in HIP.
 *
 * The method is the one of Pattabiraman et al., "A Parallel Monte Carlo Code
 * for Simulating Collisional N-body Systems" (arXiv:1206.5878), Sec. 2.1: with
 * the stars sorted by radius, (1) compute the potential, (2) fix the shared
 * timestep, (3) relax neighbouring pairs by a representative two-body
 * encounter, (5) draw a new orbit and radius for every star, (6) sort by
 * radius.  Units: G = 1, total mass 1 (Henon units).  Stars are 0-based.
 *
 * Conventions for every call:
 *  - All pointers inside cmc_state, and every pointer named *_dev, are DEVICE
 *    memory owned by the caller.  The library never allocates, frees or
 *    synchronises; each call only enqueues kernels on `stream` (a hipStream_t,
 *    NULL = the default stream) and returns.
 *  - The active star count lives on the device (cmc_scalars.n), so a sequence
 *    of calls never needs a host round trip.  `cap` bounds it.
 *  - Return value: CMC_OK, or a negative CMC_E* code when the arguments fail
 *    the host-side checks (nothing is enqueued then) or a launch fails.
 *  - Problems found on the device set sticky CMC_ST_* bits in
 *    cmc_scalars.status; the caller reads them after synchronising.
 *  - Calls on different states may run concurrently on different streams;
 *    calls on one state must be ordered (one stream).
 *  - No C++ exception crosses this boundary.
 */
#ifndef CMC_H
#define CMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CMC_ABI_VERSION 7

/* ---- return codes --------------------------------------------------------- */
#define CMC_OK 0
#define CMC_EINVAL (-1)     /* null pointer, cap out of range, bad argument    */
#define CMC_EWORKSPACE (-2) /* work_bytes < cmc_workspace_bytes(cap)            */
#define CMC_EHIP (-3)       /* a kernel launch failed (hipGetLastError)         */
#define CMC_ERANGE (-4)     /* n > cap                                          */
#define CMC_ESCRATCH (-5)   /* cmc_step_noalloc: cmc_workspace_bytes(cap) is
                               larger than CMC_SCRATCH_BYTES                    */

/* ---- sticky device status bits (cmc_scalars.status) ----------------------- */
#define CMC_ST_NONFINITE 0x01u /* a non-finite radius or velocity was produced  */
#define CMC_ST_TRIAL_CAP 0x02u /* a star used trial_cap rejection trials         */
#define CMC_ST_BOUND 0x04u     /* a trial exceeded the rejection bound F         */
#define CMC_ST_ESCAPER 0x08u   /* a star had E >= 0 and was removed              */
#define CMC_ST_DT_DEGEN 0x10u  /* no positive dt reaches the target; dt = 0     */
#define CMC_ST_NUMERIC 0x20u   /* degenerate orbit: infinite rejection bound     */
#define CMC_ST_DT_NOCONV 0x40u /* the dt solve ran out of iterations            */

/* ---- arithmetic of a call --------------------------------------------------- */
#define CMC_FP64 0  /* every step in double precision                          */
#define CMC_MIXED 1 /* fp32 pair terms, kicks and rejection trials (23-bit
                       uniforms); fp32 m/r in the potential with fp64 sums;
                       fp64 table, turning points and Q.  Results differ
                       from CMC_FP64 at ~1e-7 relative, and an accept/reject
                       decision within that of its threshold may flip.          */

/* Random numbers of a step (cmc_params.rng).  Every draw is one block of four
 * 32-bit words: the pair's first star draws one per relaxation, a star one per
 * rejection trial and one for the sign of its new v_r. */
#define CMC_RNG_PHILOX 0  /* Philox4x32-10 (Salmon et al. 2011), counter
                             (star id, step, purpose, trial): stateless       */
#define CMC_RNG_LFSR113 1 /* the generator of Sec. 3.6: L'Ecuyer's combined
                             Tausworthe LFSR113, one stream per star, the next
                             four outputs of the drawing star's stream; the
                             state (cmc_state.rng) moves with the star       */

/* Initial models of cmc_init_model (and of the ensemble) */
#define CMC_MODEL_PLUMMER 0 /* Plummer sphere (Sec. 2.1 opening paragraph)      */
#define CMC_MODEL_KING 1    /* King (1966) model with central potential W0     */

/* Device-resident scalars of one cluster (128 bytes, caller-owned). */
typedef struct cmc_scalars {
  int64_t n;          /* active star count (cmc_init_*, cmc_sort, cmc_step)     */
  double dt;          /* timestep: solved by cmc_timestep, read by cmc_relax    */
  uint32_t status;    /* sticky CMC_ST_* bits                                   */
  uint32_t dt_iters;  /* Newton iterations the last dt solve used               */
  int64_t n_esc;      /* escapers found by the last orbit pass                  */
  int64_t trials;     /* rejection trials of the last orbit pass                */
  int64_t violations; /* trials with g(s) > F in the last orbit pass            */
  int64_t capped;     /* stars that hit trial_cap in the last orbit pass        */
  double e_esc;       /* sum of m E over the last orbit pass's escapers         */
  double mass_norm;   /* total raw mass drawn by cmc_init_*                     */
  int64_t step;       /* steps taken with cmc_params.step == CMC_STEP_DEVICE    */
  int64_t corr_n;     /* stars of the last step's orbit pass whose energy
                         correction is pending (0: none; see cmc_energy_correction) */
  int64_t corr_skipped; /* stars the last correction call left unchanged (0 when
                           it found no correction pending)                      */
  int64_t reserved[4];
} cmc_scalars;

/* One cluster.  Every array has `cap` entries of device memory (rng: 4 cap
 * words).
 *  r, vr, vt, m, id : the stars, sorted by r on entry to cmc_potential,
 *                     cmc_timestep, cmc_relax and cmc_orbit (SoA).
 *  m                : double, or float when m_f32 != 0.
 *  id               : persistent star id; it names the star's random streams.
 *  phi, mcum, ssuf  : the potential table written by cmc_potential:
 *                     mcum[k] = sum_{i<=k} m_i, ssuf[k] = sum_{i>k} m_i/r_i,
 *                     phi[k] = -(mcum[k]/r[k] + ssuf[k]).
 *  r_new            : new radius from cmc_orbit, +inf for an escaper; the key
 *                     that cmc_sort orders by.
 *  sc               : device scalars (see cmc_scalars).
 *  rng              : NULL, or each star's LFSR113 state (4 words, the
 *                     component words z1..z4) in the order of the stars; when
 *                     present it moves with its star in every sort.  Needed by
 *                     steps with CMC_RNG_LFSR113.  cmc_init_* do not set it:
 *                     seed it with cmc_rng_seed_lfsr113 after the model.
 *  work, work_bytes : scratch of at least cmc_workspace_bytes(cap) bytes,
 *                     256-byte aligned; calls leave nothing in it that a later
 *                     call relies on, except the potential table a cmc_step
 *                     or cmc_potential builds for the same step's orbit pass,
 *                     and the data of a pending energy correction (see
 *                     cmc_energy_correction). */
typedef struct cmc_state {
  int64_t cap;
  double *r, *vr, *vt;
  void *m;
  int32_t m_f32;
  int32_t reserved0;
  uint32_t *id;
  double *phi, *mcum, *ssuf;
  double *r_new;
  cmc_scalars *sc;
  void *work;
  size_t work_bytes;
  uint32_t *rng;
} cmc_state;

/* Parameters of one step. */
#define CMC_STEP_DEVICE 0xFFFFFFFFu

typedef struct cmc_params {
  uint64_t seed;       /* Philox key                                              */
  uint32_t step;       /* step index: Philox counter word 1; CMC_STEP_DEVICE: use
                          sc->step and advance it (for calls replayed from a
                          captured hipGraph)                                      */
  int32_t precision;   /* CMC_FP64 or CMC_MIXED                                   */
  double gamma;        /* Coulomb logarithm ln(gamma N), N = active stars         */
  double target;       /* mean sin^2(beta/2) over pairs that fixes dt (0.03)      */
  double bound_factor; /* rejection bound F = bound_factor * max endpoint g (1.2) */
  int32_t trial_cap;   /* rejection trials per star before giving up (10000)      */
  int32_t dt_iters;    /* Newton iterations enqueued for dt; 0 = default (10)     */
  int32_t energy_corr; /* 1: potential-change energy correction (cmc_step)        */
  int32_t rng;         /* CMC_RNG_PHILOX or CMC_RNG_LFSR113 (needs s->rng)        */
} cmc_params;

/* Bytes of scratch a state of capacity `cap` needs. */
size_t cmc_workspace_bytes(int64_t cap);

/* Initial Plummer model (Sec. 2.1 opening paragraph: sample (m, r, vr, vt),
 * keep |r|, vr, vt, start sorted).  Star i < n draws from Philox key `seed`,
 * counter (i, 0, purpose, trial): r = (X1^(-2/3) - 1)^(-1/2); speed by
 * rejection on q^2 (1-q^2)^(7/2); isotropic direction; Henon-unit scaling
 * r * 3pi/16, v * sqrt(16/(3pi)).  mass_spectrum 0: m = 1/n; 1: broken power
 * law dN/dm ~ m^-1.3 on [0.1,0.5], m^-2.3 on [0.5,100], rescaled to sum 1.
 * Writes r, vr, vt, m, id sorted by radius (ties by id) and sc->n = n, clears
 * the other scalars.  CMC_ERANGE if n > cap. */
int cmc_init_plummer(cmc_state *s, int64_t n, uint64_t seed, int32_t mass_spectrum,
                     void *stream);

/* Initial model by kind: CMC_MODEL_PLUMMER as cmc_init_plummer, or
 * CMC_MODEL_KING (King 1966, central potential w0 in (0, 16]; the paper
 * names no initial model besides Plummer, so this one follows King's
 * definition).  King: in units G = sigma = r_K = 1, W'' + 2W'/r =
 * -9 rho(W)/rho(W0) with rho(W) = e^W erf(sqrt W) - sqrt(4W/pi)(1 + 2W/3)
 * and M(r) = -r^2 W', integrated by RK4 in ln r (step 0.005, series start at
 * r = 1e-4) until W = 0; r from the inverse of M(r), linear between the RK4
 * nodes; speed by rejection on v^2 (e^(W - v^2/2) - 1), v < sqrt(2W), bounded
 * by 2 e^(W-1) (W >= 1) or 2W; isotropic direction; scaled to G = M = 1,
 * E = -1/4 with E = W_pot/2 (W_pot by the trapezoid rule over the nodes).
 * Philox purposes and counters as for Plummer.  Masses as mass_spectrum.
 * CMC_EINVAL for an unknown model or w0 out of range. */
int cmc_init_model(cmc_state *s, int64_t n, uint64_t seed, int32_t model, int32_t mass_spectrum,
                   double w0, void *stream);

/* Sort (Sec. 2.1 step 6): order the stars by r_new ascending (key = bit
 * pattern of r_new + 0.0, so +inf and NaN go last), equal keys in their
 * present order; write r = r_new, vr, vt, m, id permuted accordingly and drop
 * the stars whose key is not finite (escapers) by lowering sc->n. */
int cmc_sort(cmc_state *s, void *stream);

/* Potential (Sec. 2.1 step 1): for r_k <= r < r_{k+1},
 * Phi(r) = -(1/r) sum_{i<=k} m_i - sum_{i>k} m_i/r_i.  Writes mcum, ssuf, phi
 * for the sc->n sorted stars.  precision: CMC_FP64 or CMC_MIXED. */
int cmc_potential(cmc_state *s, int32_t precision, void *stream);

/* Shared timestep (Sec. 2.1 step 2 and Sec. 3.2 bins, as fixed for this
 * method): pairs (2j, 2j+1); local density from the pair's 20-star bin;
 * t_p = (pi/32) w^3 / (ln(gamma N) n_b (m1+m2)^2); beta_p = min(pi,
 * (pi/2) sqrt(dt/t_p)); solve mean over pairs with w > 0 of sin^2(beta_p/2)
 * = p->target for dt (Newton on ln dt, started from sc->dt when > 0).
 * Writes sc->dt, sc->dt_iters; CMC_ST_DT_DEGEN / CMC_ST_DT_NOCONV bits. */
int cmc_timestep(cmc_state *s, const cmc_params *p, void *stream);

/* Two-body relaxation (Sec. 2.1 step 3(i)): rotate each pair's relative
 * velocity by beta_p (with dt = sc->dt) about a random azimuth in the
 * centre-of-mass frame; pair momentum and kinetic energy are conserved.
 * Updates vr, vt in place.  An odd last star is left alone. */
int cmc_relax(cmc_state *s, const cmc_params *p, void *stream);

/* New orbits (Sec. 2.1 step 5): E = phi_i + (vr^2+vt^2)/2, J = r_i vt_i;
 * bracket rmin and rmax between table radii by bisection on
 * Q(r) = 2E - 2Phi(r) - J^2/r^2, solve inside the bracket, then draw the new
 * radius with probability proportional to dr/|v_r| by rejection in
 * r = r_c + r_a sin s (trial j of star i uses Philox counter
 * (id_i, step, 0x30, j)).  Writes r_new (+inf when E >= 0) and the new vr,
 * vt in place; counters in sc.  Needs the table of cmc_potential. */
int cmc_orbit(cmc_state *s, const cmc_params *p, void *stream);

/* One whole step: potential -> timestep -> relax -> orbit -> sort.  The
 * potential table is kept in the workspace; phi, mcum, ssuf and r_new of the
 * state are not written (call cmc_potential for them).  With p->energy_corr
 * = 1 the step first applies the correction pending from the step before
 * (cmc_energy_correction, right after its potential) and leaves its own
 * pending; with 0 it leaves none (and a pending one is dropped unapplied).  The sort's result is
 * that of cmc_sort; for cap <= CMC_BUCKET_CAP_MAX it starts from where the orbit
 * pass found each new radius among the old ones (a counting sort on that
 * position, then each run of equal position sorted by radius), above it it is
 * cmc_sort's radix sort. */
#define CMC_BUCKET_CAP_MAX (16383LL * 2048 - 1)
int cmc_step(cmc_state *s, const cmc_params *p, void *stream);

/* cmc_step that also records events[0] on `stream` before the step and
 * events[1..5] after its potential, timestep, relax, orbit and sort phases,
 * for per-phase timing (with energy_corr, the correction and the radial
 * index of the orbit pass count to the potential phase).  events: 6
 * hipEvent_t created by the caller. */
int cmc_step_timed(cmc_state *s, const cmc_params *p, void *const *events, void *stream);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): cmc_step
 * with the library's own scratch in place of s->work.  s->work and
 * s->work_bytes are ignored (they may be NULL and 0); every other array of
 * the state is the caller's, as for cmc_step, and the result is cmc_step's
 * bit for bit.
 *  - The scratch is one static device array of CMC_SCRATCH_BYTES per GPU
 *    (64 MiB), held from the first call on that GPU until the process ends;
 *    its device address is looked up once per GPU, on the first call made
 *    while that GPU is current.  `stream` must belong to the current device.
 *  - Capacity limit: cmc_workspace_bytes(s->cap) <= CMC_SCRATCH_BYTES, about
 *    238,000 stars (about 282 bytes per star); a larger cap returns
 *    CMC_ESCRATCH and enqueues nothing.
 *  - p->energy_corr must be 0 (CMC_EINVAL otherwise): a pending correction's
 *    data would have to outlive the call in scratch that the next call on the
 *    GPU overwrites.  Like cmc_step with energy_corr = 0, the step drops a
 *    correction the state had pending.
 *  - Every call on one GPU shares that GPU's array, and each call leaves its
 *    contents behind; no call relies on what an earlier one left.  Calls that
 *    overlap in time on one GPU (different streams, or threads) race on it
 *    and give undefined results: order them on one stream.
 *  - Allocates nothing: no hipMalloc, hipFree or allocating library call. */
#define CMC_SCRATCH_BYTES ((size_t)64 << 20)
int cmc_step_noalloc(cmc_state *s, const cmc_params *p, void *stream);

/* Energy correction (Sec. 2.1 item 6): the orbits of a step are drawn in the
 * old potential Phi_old; once the stars have moved, the potential is
 * Phi_new.  Taking the potential to change linearly over the step, each star
 * that the last cmc_step (with energy_corr = 1) moved from r_old to r_new
 * gains kinetic energy per unit mass dT = (dPhi(r_old) - dPhi(r_new)) / 2,
 * dPhi = Phi_new - Phi_old, applied by scaling vr and vt by
 * sqrt(1 + 2 dT / v^2) (vr/vt unchanged).  A star with v^2 + 2 dT <= 0, or
 * v = 0 and dT != 0, keeps its velocities; sc->corr_skipped counts them.
 * Needs the table of cmc_potential of the state that step left; does
 * nothing when no correction is pending (sc->corr_n = 0) and clears it
 * after.  The data of a pending correction (old radius and potentials, the
 * sort's permutation) lives in the workspace; cmc_init_*, cmc_sort and a step
 * without energy_corr drop it.  Every star's energy moves to the one the
 * trapezoid rule gives, so apart from escapers and skipped stars the step
 * conserves T + W exactly (the shell interaction is symmetric). */
int cmc_energy_correction(cmc_state *s, void *stream);

/* Diagnostics of the sorted state and its table (needs cmc_potential):
 * out_dev[0..CMC_DIAG_N-1] = T, W = sum m phi / 2, E = T + W, 2T/|W|, M, the
 * radii holding 1%, 10%, 50%, 90% of the mass, and the core of the paper's
 * core-collapse runs (Sec. 4, after Casertano & Hut 1985): with rho_i the
 * mass of the 5 stars strictly inside the window of 7 consecutive radii
 * a..a+6, a = clamp(i-3, 0, n-7), over the shell volume between r_a and
 * r_(a+6) (windows of zero volume left out), out_dev[9] = the density-weighted
 * core radius sum rho_i r_i / sum rho_i and out_dev[10] = the core density
 * sum rho_i^2 / sum rho_i; both NaN when n < 7. */
#define CMC_DIAG_N 11
int cmc_diagnostics(const cmc_state *s, double *out_dev, void *stream);

/* Raw Philox4x32-10 blocks: out_dev[4i..4i+3] = Philox(key, ctr_dev[4i..4i+3])
 * for i < n.  The generator every random draw above goes through by default. */
int cmc_philox(uint64_t key, const uint32_t *ctr_dev, uint32_t *out_dev, int64_t n,
               void *stream);

/* LFSR113 streams (Sec. 3.6): s->rng[j] = the seed state z0 (4 words, host
 * memory, read during the call) advanced by (stream_base + id_j) * 2^80
 * steps, for j < sc->n.  The paper jumps by D = 2^80 to give each processor
 * its own stream; here each star has one.  Stream indices must stay below
 * 2^33 (= 2^113 / 2^80) for streams not to overlap: give the clusters of an
 * ensemble disjoint ranges through stream_base.  CMC_EINVAL when s->rng is
 * NULL, a component of z0 has its top k bits all zero (k = 31, 29, 28, 25:
 * z1 < 2, z2 < 8, z3 < 16, z4 < 128), or stream_base >= 2^33. */
int cmc_rng_seed_lfsr113(cmc_state *s, const uint32_t *z0, uint64_t stream_base, void *stream);

/* Raw LFSR113 words: for each of the n states state_dev[4i..4i+3],
 * out_dev[4(i blocks + b) .. +3] = its block b < blocks (4 consecutive
 * outputs).  The states are not changed. */
int cmc_lfsr113(const uint32_t *state_dev, uint32_t *out_dev, int64_t n, int32_t blocks,
                void *stream);

/* ---- ensembles ----------------------------------------------------------------
 * Independent clusters of uneven N advanced together: every kernel of a step
 * is one launch over all clusters (a per-launch map gives each block its
 * cluster), per-cluster reductions, Delta t solves, potential scans and sorts
 * never cross a cluster, and each cluster keeps its own state arrays and
 * workspace (a cmc_state each, as for the single-cluster calls).  Sec. 2.1's
 * step applies to each cluster unchanged; the ensemble is this library's
 * batching of it. */

/* What cluster c of an ensemble starts as and relaxes with. */
typedef struct cmc_cluster_spec {
  int64_t n;             /* stars of the initial model (<= the state's cap)      */
  uint64_t seed;         /* the cluster's Philox key                             */
  double gamma;          /* Coulomb logarithm ln(gamma N) of the cluster         */
  int32_t model;         /* CMC_MODEL_PLUMMER or CMC_MODEL_KING                  */
  int32_t mass_spectrum; /* 0 or 1, as cmc_init_plummer                          */
  double w0;             /* King central potential                               */
} cmc_cluster_spec;

#define CMC_SHAPES 24

/* Host handle of an ensemble, filled by cmc_batch_prepare.  `dev` is device
 * memory of cmc_batch_device_bytes() bytes, 256-byte aligned, owned by the
 * caller; it holds the cluster table and the launch maps. */
typedef struct cmc_batch {
  int32_t clusters;
  int32_t m_f32;                /* mass storage (every cluster alike)            */
  void *dev;
  size_t dev_bytes;
  int64_t total[CMC_SHAPES];    /* blocks per launch shape over all clusters     */
  int32_t top_entries;          /* LDS entries of the orbit table's top levels   */
  int32_t bucket_sort;          /* 1: the step sorts by buckets (every capacity  */
                                /*    <= CMC_BUCKET_CAP_MAX), 0: radix sort      */
  int32_t lfsr_ready;           /* 1: every cluster has an rng array             */
  int32_t sorted_searches;      /* the launch table's choice for the ensemble    */
} cmc_batch;

/* Device bytes of the ensemble tables for these states (0 if invalid). */
size_t cmc_batch_device_bytes(const cmc_state *states, int32_t clusters);

/* Checks the states and specs (CMC_EINVAL / CMC_EWORKSPACE / CMC_ERANGE as the
 * single-cluster calls; masses must be all f32 or all f64; clusters in
 * [1, 65535]), fills *b and copies the tables into `dev`.  A setup call: it
 * blocks until the copy is done (hipMemcpy), so it is not capturable.  The
 * states' arrays must stay where they are for as long as b is used. */
int cmc_batch_prepare(cmc_batch *b, const cmc_state *states, const cmc_cluster_spec *specs,
                      int32_t clusters, void *dev, size_t dev_bytes);

/* Initial model of every cluster (as cmc_init_model with its spec). */
int cmc_batch_init(const cmc_batch *b, void *stream);

/* One step of every cluster (as cmc_step); p->seed and p->gamma are ignored
 * (each cluster has its own); CMC_RNG_LFSR113 needs b->lfsr_ready.  With p->step == CMC_STEP_DEVICE the step index
 * is each cluster's sc->step, advanced at the end: a call captured once in a
 * hipGraph then advances the ensemble each time the graph is replayed. */
int cmc_batch_step(const cmc_batch *b, const cmc_params *p, void *stream);

/* The step's phases one at a time over every cluster, each as its
 * single-cluster call on each cluster (Sec. 2.1 applied per cluster); the
 * cluster's own seed and gamma are used, p->seed and p->gamma are ignored;
 * CMC_RNG_LFSR113 needs b->lfsr_ready.  Called in the order potential,
 * timestep, relax, orbit, sort they give the result of one cmc_batch_step
 * (without energy_corr) bit for bit.
 *  cmc_batch_sort     : as cmc_sort (step 6): order by r_new, drop escapers.
 *  cmc_batch_potential: as cmc_potential (step 1); below.
 *  cmc_batch_timestep : as cmc_timestep (step 2): each cluster's sc->dt.
 *  cmc_batch_relax    : as cmc_relax (step 3(i)) with each cluster's sc->dt.
 *  cmc_batch_orbit    : as cmc_orbit (step 5): needs cmc_batch_potential's
 *                       public table; writes r_new, vr, vt. */
int cmc_batch_sort(const cmc_batch *b, void *stream);
int cmc_batch_timestep(const cmc_batch *b, const cmc_params *p, void *stream);
int cmc_batch_relax(const cmc_batch *b, const cmc_params *p, void *stream);
int cmc_batch_orbit(const cmc_batch *b, const cmc_params *p, void *stream);

/* cmc_potential of every cluster (public phi, mcum, ssuf). */
int cmc_batch_potential(const cmc_batch *b, int32_t precision, void *stream);

/* cmc_energy_correction of every cluster (needs cmc_batch_potential). */
int cmc_batch_energy_correction(const cmc_batch *b, void *stream);

/* cmc_diagnostics of every cluster: out_dev[CMC_DIAG_N c .. CMC_DIAG_N c +
 * CMC_DIAG_N - 1] for cluster c. */
int cmc_batch_diagnostics(const cmc_batch *b, double *out_dev, void *stream);

/* ---- launch table ------------------------------------------------------------
 * How the orbit pass (Sec. 2.1 item 5) is launched, by capacity: a read-only
 * table that the library consults when it sets up a call (each single-cluster
 * call, and cmc_batch_prepare for an ensemble, with the capacity of its
 * largest cluster).  Every entry gives the same results bit for bit; only the
 * speed differs.  The built-in table holds measured defaults; an autotuner
 * (the package's tune.py, after the paper's own launch-configuration study,
 * Appendix A) times candidates on the GPU and installs its table here.
 *  sorted         : 1: the turning-point searches are grouped by the sample
 *                   of the LDS-resident top levels they reach, so that the
 *                   searches sharing a subtree run together (where a group
 *                   spans at most 4096 stars, capacities up to about 1.06e7,
 *                   its block holds the whole subtree in LDS); 0: each star's
 *                   wavefront searches its own brackets to the bottom.
 *  bracket_blocks : resident blocks of the direct search kernel for a single
 *                   cluster (an ensemble shares them out by capacity), 8..65535.
 *  trial_chunk    : stars per wavefront chunk of the rejection-trial kernel,
 *                   a multiple of 64 in [64, 1024]. */
typedef struct cmc_tuning {
  int64_t min_cap;        /* the entry serves capacities >= min_cap          */
  int32_t sorted;
  int32_t bracket_blocks;
  int32_t trial_chunk;
  int32_t reserved[3];
} cmc_tuning;
#define CMC_TUNING_MAX 32

/* Install a launch table of n entries (n <= CMC_TUNING_MAX, min_cap strictly
 * increasing, the first 0); n = 0 restores the built-in table.  The table is
 * copied.  A setup call: not to be made while other calls of the library run
 * or are being set up in other threads.  CMC_EINVAL for a bad table (the
 * table in use is then unchanged). */
int cmc_set_tuning(const cmc_tuning *entries, int32_t n);

/* The entry of the table in use that serves capacity cap (*out). */
int cmc_get_tuning(int64_t cap, cmc_tuning *out);

/* Text for a CMC_E* code. */
const char *cmc_strerror(int code);

/* CMC_ABI_VERSION of the loaded library. */
int cmc_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif

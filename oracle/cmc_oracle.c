/*
 * cmc_oracle.c -- plain FP64 CPU oracle of one Henon Monte Carlo step.
 *
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline).  Shares no
 * code with the HIP library.  See cmc_oracle.h for the interface and the
 * paper reference.  Built with -ffp-contract=off so every line is the IEEE
 * operation it reads as.  Built a second time with OpenMP for the CPU
 * baseline's all-core timing: the per-star and per-pair loops are
 * independent, and every sum runs serially in index order, so both builds
 * give the same results bit for bit; the scan and the sort stay serial.
 */
#include "cmc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* Compensated (Neumaier) summation.                                          */
typedef struct {
  double s, c;
} ksum;

static void kadd(ksum *k, double x) {
  double t = k->s + x;
  if (fabs(k->s) >= fabs(x))
    k->c += (k->s - t) + x;
  else
    k->c += (x - t) + k->s;
  k->s = t;
}

static double kval(const ksum *k) { return k->s + k->c; }

/* ------------------------------------------------------------------------- */
/* Philox4x32-10, from its definition in Salmon et al. (SC'11): ten rounds of
 * two 32x32->64 multiplies whose halves are xor-ed with the other two counter
 * words and the key; the key is bumped by two Weyl constants between rounds. */
void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t mul0 = 0xD2511F53u, mul1 = 0xCD9E8D57u;
  const uint32_t weyl0 = 0x9E3779B9u, weyl1 = 0xBB67AE85u;
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)mul0 * (uint64_t)x0;
    uint64_t p1 = (uint64_t)mul1 * (uint64_t)x2;
    uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)p1;
    uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)p0;
    x0 = y0;
    x1 = y1;
    x2 = y2;
    x3 = y3;
    k0 += weyl0;
    k1 += weyl1;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

/* Threads the library's parallel loops use: 1 unless built with OpenMP. */
int ora_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void ora_philox_many(int64_t n, uint64_t key, const uint32_t *ctr, uint32_t *out) {
  uint32_t k[2] = {(uint32_t)key, (uint32_t)(key >> 32)};
  for (int64_t i = 0; i < n; ++i) ora_philox4x32_10(ctr + 4 * i, k, out + 4 * i);
}

double ora_u01(uint32_t hi, uint32_t lo) {
  uint64_t x = (((uint64_t)hi << 32) | (uint64_t)lo) >> 12; /* 52 bits */
  return ((double)(2 * x + 1)) * 0x1.0p-53;
}

float ora_u01f(uint32_t hi) {
  uint32_t x = hi >> 9; /* 23 bits */
  return ((float)(2 * x + 1)) * 0x1.0p-24f;
}

static void draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                 uint32_t w[4]) {
  uint32_t ctr[4] = {c0, c1, c2, c3};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  ora_philox4x32_10(ctr, key, w);
}

/* ------------------------------------------------------------------------- */
/* The generator of Sec. 3.6: L'Ecuyer's combined Tausworthe LFSR113 (Math.
 * Comp. 68, 1999).  Four component LFSRs of degrees k = 31, 29, 28, 25 with
 * (q, s) = (6, 18), (2, 2), (13, 7), (3, 13); a component's state is the top
 * k bits of its word, one step is
 *   b = ((z << q) ^ z) >> (k - s);   z = ((z & top k bits) << s) ^ b,
 * and each output is the XOR of the four words.  Period about 2^113.  A step
 * is linear over GF(2) in the word, so D steps are the D-th power of a 32x32
 * bit matrix, kept as its 32 columns (the image of each bit). */
static const int lfsr_k[4] = {31, 29, 28, 25};
static const int lfsr_q[4] = {6, 2, 13, 3};
static const int lfsr_s[4] = {18, 2, 7, 13};

static uint32_t lfsr_comp(uint32_t z, int c) {
  const uint32_t top = ~0u << (32 - lfsr_k[c]);
  const uint32_t b = ((z << lfsr_q[c]) ^ z) >> (lfsr_k[c] - lfsr_s[c]);
  return ((z & top) << lfsr_s[c]) ^ b;
}

uint32_t ora_lfsr113_next(uint32_t z[4]) {
  for (int c = 0; c < 4; ++c) z[c] = lfsr_comp(z[c], c);
  return z[0] ^ z[1] ^ z[2] ^ z[3];
}

void ora_lfsr113_block(uint32_t z[4], uint32_t w[4]) {
  for (int i = 0; i < 4; ++i) w[i] = ora_lfsr113_next(z);
}

static void lfsr_matrix(int c, uint32_t col[32]) {
  for (int i = 0; i < 32; ++i) col[i] = lfsr_comp(1u << i, c);
}

static uint32_t mat_apply(const uint32_t col[32], uint32_t v) {
  uint32_t r = 0;
  for (int i = 0; i < 32; ++i)
    if ((v >> i) & 1u) r ^= col[i];
  return r;
}

static void mat_square(uint32_t col[32]) {
  uint32_t t[32];
  for (int i = 0; i < 32; ++i) t[i] = mat_apply(col, col[i]);
  memcpy(col, t, sizeof t);
}

void ora_lfsr113_jump_pow2(uint32_t z[4], int e) {
  for (int c = 0; c < 4; ++c) {
    uint32_t col[32];
    lfsr_matrix(c, col);
    for (int t = 0; t < e; ++t) mat_square(col);
    z[c] = mat_apply(col, z[c]);
  }
}

void ora_lfsr113_stream(const uint32_t z0[4], uint64_t id, uint32_t z[4]) {
  for (int c = 0; c < 4; ++c) {
    uint32_t col[32];
    lfsr_matrix(c, col);
    for (int t = 0; t < 80; ++t) mat_square(col); /* one stream: 2^80 steps */
    uint32_t v = z0[c];
    for (uint64_t x = id; x; x >>= 1) {
      if (x & 1u) v = mat_apply(col, v);
      mat_square(col);
    }
    z[c] = v;
  }
}

int64_t ora_lfsr113_component_period(int c, uint32_t z, int64_t limit) {
  const uint32_t top = ~0u << (32 - lfsr_k[c]);
  const uint32_t start = z & top;
  for (int64_t t = 1; t <= limit; ++t) {
    z = lfsr_comp(z, c);
    if ((z & top) == start) return t;
  }
  return -1;
}

/* Where a step's random blocks come from: Philox keyed by the seed with
 * counter (star id, step, purpose, trial), or, with lfsr set, the next block
 * of the star's own LFSR113 stream (4 state words per star, in the order of
 * the arrays).  consume = 0 reads a block without advancing the stream. */
typedef struct {
  uint64_t seed;
  uint32_t step;
  uint32_t *lfsr;
} draws;

static void star_draw(const draws *d, const uint32_t *id, int64_t k, uint32_t purpose,
                      uint32_t trial, int consume, uint32_t w[4]) {
  if (!d->lfsr) {
    draw(d->seed, id[k], d->step, purpose, trial, w);
    return;
  }
  uint32_t z[4];
  memcpy(z, d->lfsr + 4 * k, sizeof z);
  ora_lfsr113_block(z, w);
  if (consume) memcpy(d->lfsr + 4 * k, z, sizeof z);
}

/* ------------------------------------------------------------------------- */
/* Initial Plummer model.  The paper samples (m, r, vr, vt) from a
 * distribution function and keeps only |r|, vr and vt (Sec. 2.1, opening
 * paragraph).  Plummer sphere with scale radius 1: r = (X1^(-2/3) - 1)^(-1/2);
 * speed v = q sqrt(2) (1+r^2)^(-1/4) with q drawn by rejection on
 * q^2 (1-q^2)^(7/2) under the bound 0.1; isotropic direction cos(theta) =
 * 2 X6 - 1.  Then Henon units: r * 3pi/16, v * sqrt(16/(3pi)). */
/* Masses: 1/n each, or the broken power law dN/dm ~ m^-1.3 on [0.1,0.5],
 * m^-2.3 on [0.5,100] (continuous at 0.5; segment weights from the
 * integrals), drawn by inverse CDF per segment and divided by their sum. */
static void draw_masses(int64_t n, uint64_t seed, int mass_spectrum, double *m) {
  if (!mass_spectrum) {
    for (int64_t i = 0; i < n; ++i) m[i] = 1.0 / (double)n;
    return;
  }
  const double ma = 0.1, mb = 0.5, mc = 100.0;
  const double ia = (pow(ma, -0.3) - pow(mb, -0.3)) / 0.3;
  const double ib = 0.5 * (pow(mb, -1.3) - pow(mc, -1.3)) / 1.3;
  const double f1 = ia / (ia + ib);
  ksum total = {0.0, 0.0};
  for (int64_t i = 0; i < n; ++i) {
    uint32_t w[4];
    draw(seed, (uint32_t)i, 0u, ORA_P_INIT_MASS, 0u, w);
    double us = ora_u01(w[1], w[0]);
    double um = ora_u01(w[3], w[2]);
    double mm;
    if (us < f1) {
      double lo = pow(ma, -0.3), hi = pow(mb, -0.3);
      mm = pow(lo - um * (lo - hi), -1.0 / 0.3);
    } else {
      double lo = pow(mb, -1.3), hi = pow(mc, -1.3);
      mm = pow(lo - um * (lo - hi), -1.0 / 1.3);
    }
    m[i] = mm;
    kadd(&total, mm);
  }
  double tot = kval(&total);
  for (int64_t i = 0; i < n; ++i) m[i] = m[i] / tot;
}

void ora_plummer(int64_t n, uint64_t seed, int mass_spectrum, double *r, double *vr,
                 double *vt, double *m, uint32_t *id) {
  const double rscale = 3.0 * PI / 16.0;
  const double vscale = sqrt(16.0 / (3.0 * PI));
  for (int64_t i = 0; i < n; ++i) {
    uint32_t w[4];
    draw(seed, (uint32_t)i, 0u, ORA_P_INIT_POS, 0u, w);
    double x1 = ora_u01(w[1], w[0]);
    double x6 = ora_u01(w[3], w[2]);
    /* (X^(-2/3) - 1)^(-1/2) = sqrt(y / (1 - y)), y = X^(2/3); 1 - y via expm1
     * so the far tail keeps full relative precision. */
    double lx = (2.0 / 3.0) * log(x1);
    double y = exp(lx);
    double omy = -expm1(lx);
    double rr = sqrt(y / omy);

    double q = 0.0;
    for (uint32_t j = 0; j < 1000000u; ++j) {
      draw(seed, (uint32_t)i, 0u, ORA_P_INIT_SPEED, j, w);
      q = ora_u01(w[1], w[0]);
      double x5 = ora_u01(w[3], w[2]);
      double t = 1.0 - q * q;
      double g = q * q * (t * t * t) * sqrt(t);
      if (0.1 * x5 < g) break;
    }
    double v = q * sqrt(2.0) * pow(1.0 + rr * rr, -0.25);
    double c = 2.0 * x6 - 1.0;
    double s = sqrt((1.0 - c) * (1.0 + c));

    r[i] = rr * rscale;
    vr[i] = v * vscale * c;
    vt[i] = v * vscale * s;
    id[i] = (uint32_t)i;
  }
  draw_masses(n, seed, mass_spectrum, m);
}

/* ------------------------------------------------------------------------- */
/* King (1966) model with central potential W0 (an initial model the paper does
 * not use; the ensemble workload does).  Units G = sigma = r_K = 1: the
 * dimensionless potential W(r) solves the Poisson equation
 *   (1/r^2) d/dr (r^2 dW/dr) = -9 rho(W) / rho(W0),
 *   rho(W) = e^W erf(sqrt W) - sqrt(4W/pi) (1 + 2W/3)   (King's lowered
 *   isothermal distribution f ~ e^(W - v^2/2) - 1 integrated over v),
 * with W(0) = W0, W'(0) = 0; the enclosed mass is M(r) = -r^2 dW/dr, and the
 * tidal radius is where W reaches 0.  Integration: RK4 in t = ln r on
 * (W, U = r^2 W'), step 0.005, from r = 1e-4 where the series
 *   W = W0 - 1.5 r^2 + 0.675 a r^4,  U = -3 r^3 + 2.7 a r^5,
 *   a = rho'(W0)/rho(W0) = (e^W0 erf(sqrt W0) - sqrt(4 W0/pi)) / rho(W0),
 * holds (obtained by inserting W = W0 - 1.5 r^2 + b r^4 and
 * rho/rho0 = 1 + a (W - W0) into the equation).  The last step, in which W
 * turns non-positive, is cut at the zero of the linear interpolant of W. */
static double king_rho(double W) {
  if (!(W > 0.0)) return 0.0;
  if (W < 0.1) {
    /* e^W erf(sqrt W) = (2/sqrt pi) sqrt W sum_{j>=0} (2W)^j / (2j+1)!!; the
     * first two terms cancel against sqrt(4W/pi)(1 + 2W/3) */
    double term = 4.0 * W * W / 15.0, sum = 0.0;
    for (int j = 2; j < 12; ++j) {
      sum += term;
      term *= 2.0 * W / (2.0 * j + 3.0);
    }
    return (2.0 / sqrt(PI)) * sqrt(W) * sum;
  }
  return exp(W) * erf(sqrt(W)) - sqrt(4.0 * W / PI) * (1.0 + 2.0 * W / 3.0);
}

double ora_king_density(double W) { return king_rho(W); }

static void king_rhs(double t, double W, double U, double rho0, double *dW, double *dU) {
  double r = exp(t);
  *dW = U / r;                                 /* r dW/dr */
  *dU = -9.0 * r * r * r * king_rho(W) / rho0; /* r dU/dr */
}

int ora_king_profile(double w0, double *rk, double *Wk, double *Mk, int cap, double *tail) {
  const double h = 0.005;
  double rho0 = king_rho(w0);
  double a = (exp(w0) * erf(sqrt(w0)) - sqrt(4.0 * w0 / PI)) / rho0;
  double r = 1e-4;
  double W = w0 - 1.5 * r * r + 0.675 * a * r * r * r * r;
  double U = -3.0 * r * r * r + 2.7 * a * r * r * r * r * r;
  double t = log(r);
  int k = 0;
  rk[0] = r;
  Wk[0] = W;
  Mk[0] = -U;
  double rt = r, Mt = -U;
  while (k + 2 < cap) {
    double k1W, k1U, k2W, k2U, k3W, k3U, k4W, k4U;
    king_rhs(t, W, U, rho0, &k1W, &k1U);
    king_rhs(t + 0.5 * h, W + 0.5 * h * k1W, U + 0.5 * h * k1U, rho0, &k2W, &k2U);
    king_rhs(t + 0.5 * h, W + 0.5 * h * k2W, U + 0.5 * h * k2U, rho0, &k3W, &k3U);
    king_rhs(t + h, W + h * k3W, U + h * k3U, rho0, &k4W, &k4U);
    double Wn = W + (h / 6.0) * (k1W + 2.0 * k2W + 2.0 * k3W + k4W);
    double Un = U + (h / 6.0) * (k1U + 2.0 * k2U + 2.0 * k3U + k4U);
    if (!(Wn > 0.0)) {
      double f = W / (W - Wn);
      rt = exp(t + f * h);
      Mt = -(U + f * (Un - U));
      break;
    }
    W = Wn;
    U = Un;
    t = t + h;
    ++k;
    rk[k] = exp(t);
    Wk[k] = W;
    Mk[k] = -U;
    rt = rk[k];
    Mt = -U;
  }
  ++k;
  rk[k] = rt;
  Wk[k] = 0.0;
  Mk[k] = Mt;
  /* potential energy W_pot = -int M dM / r (G = 1), trapezoid rule in M */
  double wpot = 0.0;
  for (int q = 0; q < k; ++q)
    wpot -= 0.5 * (Mk[q] / rk[q] + Mk[q + 1] / rk[q + 1]) * (Mk[q + 1] - Mk[q]);
  tail[0] = rt;
  tail[1] = Mt;
  tail[2] = wpot;
  return k + 1;
}

/* Stars of a King model: r from the inverse of M(r) (linear between the
 * profile nodes, M = 3 r^3 inside the first node), speed by rejection from
 * v^2 (e^(W - v^2/2) - 1) on [0, sqrt(2W)] under the bound
 * max_v v^2 e^(W - v^2/2) = 2 e^(W-1) (W >= 1) or 2W (W < 1), isotropic
 * direction; then units G = M = 1 and E = W_pot/2 (virial equilibrium)
 * scaled to -1/4: lengths by s = -4 E / M_t^2, speeds by 1/sqrt(M_t s). */
#define ORA_KING_NODES 4096
void ora_king(int64_t n, uint64_t seed, double w0, int mass_spectrum, double *r, double *vr,
              double *vt, double *m, uint32_t *id) {
  double *rk = (double *)malloc(3 * ORA_KING_NODES * sizeof(double));
  double *Wk = rk + ORA_KING_NODES, *Mk = Wk + ORA_KING_NODES, tail[3];
  int nodes = ora_king_profile(w0, rk, Wk, Mk, ORA_KING_NODES, tail);
  double Mt = tail[1], wpot = tail[2];
  double s = -4.0 * (0.5 * wpot) / (Mt * Mt);
  for (int64_t i = 0; i < n; ++i) {
    uint32_t w[4];
    draw(seed, (uint32_t)i, 0u, ORA_P_INIT_POS, 0u, w);
    double x1 = ora_u01(w[1], w[0]);
    double x6 = ora_u01(w[3], w[2]);
    double target = x1 * Mt, rr, Wr;
    if (target < Mk[0]) {
      rr = cbrt(target / 3.0);
      Wr = w0 - 1.5 * rr * rr;
    } else {
      int lo = 0, hi = nodes - 1; /* Mk[lo] <= target < Mk[hi] */
      while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (Mk[mid] <= target)
          lo = mid;
        else
          hi = mid;
      }
      double f = (target - Mk[lo]) / (Mk[hi] - Mk[lo]);
      rr = rk[lo] + f * (rk[hi] - rk[lo]);
      Wr = Wk[lo] + f * (Wk[hi] - Wk[lo]);
    }
    double v = 0.0;
    if (Wr > 0.0) {
      double vmax = sqrt(2.0 * Wr);
      double bound = (Wr >= 1.0) ? 2.0 * exp(Wr - 1.0) : 2.0 * Wr;
      for (uint32_t j = 0; j < 1000000u; ++j) {
        draw(seed, (uint32_t)i, 0u, ORA_P_INIT_SPEED, j, w);
        v = vmax * ora_u01(w[1], w[0]);
        double x5 = ora_u01(w[3], w[2]);
        if (x5 * bound < v * v * expm1(Wr - 0.5 * v * v)) break;
      }
    }
    double c = 2.0 * x6 - 1.0;
    double sn = sqrt((1.0 - c) * (1.0 + c));
    double vv = v / sqrt(Mt * s);
    r[i] = rr * s;
    vr[i] = vv * c;
    vt[i] = vv * sn;
    id[i] = (uint32_t)i;
  }
  draw_masses(n, seed, mass_spectrum, m);
  free(rk);
}

/* ------------------------------------------------------------------------- */
/* Sort (Sec. 2.1 step 6): ascending radius.  The key of a radius x is the bit
 * pattern of x + 0.0 read as an unsigned integer, which orders non-negative
 * numbers and +inf numerically (escapers carry +inf and land last).  Equal
 * keys keep their previous order. */
typedef struct {
  uint64_t key;
  int64_t idx;
} kv;

static int kv_cmp(const void *pa, const void *pb) {
  const kv *a = (const kv *)pa, *b = (const kv *)pb;
  if (a->key < b->key) return -1;
  if (a->key > b->key) return 1;
  return (a->idx < b->idx) ? -1 : (a->idx > b->idx);
}

static uint64_t radius_key(double x) {
  double y = x + 0.0;
  uint64_t k;
  memcpy(&k, &y, sizeof k);
  return k;
}

void ora_sort_perm(int64_t n, const double *key, int64_t *perm) {
  kv *a = (kv *)malloc((size_t)(n > 0 ? n : 1) * sizeof(kv));
  for (int64_t i = 0; i < n; ++i) {
    a[i].key = radius_key(key[i]);
    a[i].idx = i;
  }
  qsort(a, (size_t)n, sizeof(kv), kv_cmp);
  for (int64_t i = 0; i < n; ++i) perm[i] = a[i].idx;
  free(a);
}

/* ------------------------------------------------------------------------- */
/* Potential (Sec. 2.1 step 1).  For r_k <= r < r_{k+1} the paper gives
 * Phi(r) = -G [ (1/r) sum_{i<=k} m_i + sum_{i>k} m_i / r_i ]; at the star
 * radii this is Phi_k = -(M_k / r_k + S_k) with M_k the inclusive mass prefix
 * and S_k the exclusive suffix of m_i/r_i (G = 1). */
void ora_potential(int64_t n, const double *r, const double *m, double *phi, double *mcum,
                   double *ssuf) {
  ksum M = {0.0, 0.0};
  for (int64_t k = 0; k < n; ++k) {
    kadd(&M, m[k]);
    mcum[k] = kval(&M);
  }
  ksum S = {0.0, 0.0};
  for (int64_t k = n - 1; k >= 0; --k) {
    double s = kval(&S);
    if (ssuf) ssuf[k] = s;
    phi[k] = -(mcum[k] / r[k] + s);
    kadd(&S, m[k] / r[k]);
  }
}

/* Phi inside interval k = [r_k, r_{k+1}] straight from the defining equation:
 * -(M_k / x + S_k); for k = -1 (x < r_0) the potential is flat at Phi_0.  This
 * equals the paper's interpolation linear in 1/r between Phi_k and Phi_{k+1}
 * but never subtracts two large terms. */
static double phi_in(const double *phi, const double *mcum, const double *ssuf, int64_t k,
                     double x) {
  if (k < 0) return phi[0];
  return -(mcum[k] / x + ssuf[k]);
}

/* Last table index k in [klo, khi] with r_k <= x (k = klo - 1 never: r_{-1} = 0). */
static int64_t interval_of(const double *r, int64_t klo, int64_t khi, double x) {
  int64_t lo = klo, hi = khi + 1;
  while (hi - lo > 1) {
    int64_t mid = lo + (hi - lo) / 2;
    if (r[mid] <= x)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

double ora_phi_at(int64_t n, const double *r, const double *phi, const double *mcum,
                  const double *ssuf, double x) {
  return phi_in(phi, mcum, ssuf, interval_of(r, -1, n - 1, x), x);
}

/* ------------------------------------------------------------------------- */
/* Pair geometry for relaxation (Sec. 2.1 step 3(i); bins of Sec. 3.2).
 * Neighbour pairs are (2p, 2p+1) in radial order.  The local number density
 * comes from the pair's 20-star bin [20b, 20b+19] (a short last bin is merged
 * into the previous one): n_b = (P_b - 1) / (4pi/3 (r_hi^3 - r_lo^3)).
 * The 3-D relative velocity puts star 2 at a random azimuth psi of its
 * transverse velocity.  The representative-encounter time is
 * t_p = (pi/32) w^3 / (lnL n_b (m1+m2)^2), the same combination as the
 * relaxation timestep equation with G = 1, and the deflection angle is
 * beta = min(pi, (pi/2) sqrt(dt / t_p)). */
typedef struct {
  int64_t a, b;
  double v2[3], w[3], wm, tp, nb, u2;
} pair_geo;

static void pair_geometry(int64_t n, int64_t p, const double *r, const double *m,
                          const double *vr, const double *vt, const uint32_t *id,
                          const draws *d, int consume, double lnL, pair_geo *g) {
  int64_t nbins = n / 20;
  if (nbins < 1) nbins = 1;
  int64_t a = 2 * p, b = 2 * p + 1;
  int64_t bin = a / 20;
  if (bin > nbins - 1) bin = nbins - 1;
  int64_t lo = 20 * bin;
  int64_t hi = (bin == nbins - 1) ? n - 1 : 20 * bin + 19;
  double rl = r[lo], rh = r[hi];
  double vol = (4.0 * PI / 3.0) * (rh - rl) * (rh * rh + rh * rl + rl * rl);
  double nb = (vol > 0.0) ? (double)(hi - lo) / vol : INFINITY;

  uint32_t w4[4];
  star_draw(d, id, a, ORA_P_RELAX, 0u, consume, w4); /* the pair's first star */
  double u1 = ora_u01(w4[1], w4[0]);
  double u2 = ora_u01(w4[3], w4[2]);
  double psi = 2.0 * PI * u1;

  double v2x = vr[b], v2y = vt[b] * cos(psi), v2z = vt[b] * sin(psi);
  double wx = vr[a] - v2x;
  double wy = vt[a] - v2y;
  double wz = 0.0 - v2z;
  double wm = sqrt(wx * wx + wy * wy + wz * wz);
  double ms = m[a] + m[b];
  double tp;
  if (ms == 0.0 || lnL == 0.0)
    tp = INFINITY;
  else if (isinf(nb))
    tp = 0.0;
  else
    tp = (PI / 32.0) * (wm * wm * wm) / (lnL * nb * (ms * ms));

  g->a = a;
  g->b = b;
  g->v2[0] = v2x;
  g->v2[1] = v2y;
  g->v2[2] = v2z;
  g->w[0] = wx;
  g->w[1] = wy;
  g->w[2] = wz;
  g->wm = wm;
  g->tp = tp;
  g->nb = nb;
  g->u2 = u2;
}

static double coulomb_log(double gamma, int64_t n) {
  double l = log(gamma * (double)n);
  return (l > 0.0) ? l : 0.0; /* no relaxation when gamma N <= 1 */
}

static double beta_of(double tp, double dt) {
  if (!(dt > 0.0) || isinf(tp)) return 0.0;
  if (tp == 0.0) return PI;
  double b = 0.5 * PI * sqrt(dt / tp);
  return (b < PI) ? b : PI;
}

static int64_t pair_terms_d(int64_t n, const double *r, const double *m, const double *vr,
                            const double *vt, const uint32_t *id, const draws *src,
                            double gamma, double *w, double *tp, double *nb) {
  int64_t np = n / 2;
  double lnL = coulomb_log(gamma, n);
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < np; ++p) {
    pair_geo g;
    pair_geometry(n, p, r, m, vr, vt, id, src, 0, lnL, &g);
    if (w) w[p] = g.wm;
    if (tp) tp[p] = g.tp;
    if (nb) nb[p] = g.nb;
  }
  return np;
}

int64_t ora_pair_terms(int64_t n, const double *r, const double *m, const double *vr,
                       const double *vt, const uint32_t *id, uint64_t seed, uint32_t step,
                       double gamma, double *w, double *tp, double *nb) {
  const draws d = {seed, step, NULL};
  return pair_terms_d(n, r, m, vr, vt, id, &d, gamma, w, tp, nb);
}

double ora_mean_sin2(int64_t np, const double *w, const double *tp, double dt) {
  ksum s = {0.0, 0.0};
  int64_t cnt = 0;
  double *h2 = (double *)malloc((size_t)(np > 0 ? np : 1) * sizeof(double));
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < np; ++p) {
    double h = sin(0.5 * beta_of(tp[p], dt));
    h2[p] = h * h;
  }
  for (int64_t p = 0; p < np; ++p) {
    if (!(w[p] > 0.0)) continue;
    kadd(&s, h2[p]);
    ++cnt;
  }
  free(h2);
  return cnt ? kval(&s) / (double)cnt : 0.0;
}

/* dt rule: the mean over pairs of sin^2(beta/2) equals the target.  The mean
 * is non-decreasing in dt, so bisection on x = ln dt finds the unique root. */
double ora_solve_dt(int64_t np, const double *w, const double *tp, double target,
                    uint32_t *status) {
  int64_t cnt = 0, n_zero = 0, n_inf = 0;
  for (int64_t p = 0; p < np; ++p) {
    if (!(w[p] > 0.0)) continue;
    ++cnt;
    if (tp[p] == 0.0) ++n_zero;
    if (isinf(tp[p])) ++n_inf;
  }
  /* limits: dt -> 0+ gives the share of beta = pi pairs, dt -> inf gives the
   * share of pairs that can be deflected at all */
  if (cnt == 0 || (double)n_zero / (double)cnt >= target ||
      (double)(cnt - n_inf) / (double)cnt <= target) {
    if (status) *status |= ORA_ST_DT_DEGEN;
    return 0.0;
  }
  double lo = 0.0, hi = 0.0;
  double f0 = ora_mean_sin2(np, w, tp, 1.0);
  if (f0 < target) {
    lo = 0.0;
    hi = 8.0;
    while (ora_mean_sin2(np, w, tp, exp(hi)) < target) {
      lo = hi;
      hi += 8.0;
    }
  } else {
    hi = 0.0;
    lo = -8.0;
    while (!(ora_mean_sin2(np, w, tp, exp(lo)) < target)) {
      hi = lo;
      lo -= 8.0;
    }
  }
  for (int it = 0; it < 400; ++it) {
    double mid = lo + 0.5 * (hi - lo);
    if (mid <= lo || mid >= hi) break;
    if (ora_mean_sin2(np, w, tp, exp(mid)) < target)
      lo = mid;
    else
      hi = mid;
  }
  return exp(lo + 0.5 * (hi - lo));
}

/* Two-body relaxation (Sec. 2.1 step 3(i)): rotate the pair's relative
 * velocity by beta about a random azimuth psi' in the centre-of-mass frame.
 * The frame is e1 = w/|w|, e2 = unit(e1 x a) with a the coordinate axis of the
 * smallest |w| component (lowest index on ties), e3 = e1 x e2.  Pair momentum
 * and kinetic energy are conserved exactly in real arithmetic. */
static void relax_d(int64_t n, const double *r, const double *m, double *vr, double *vt,
                    const uint32_t *id, const draws *src, double gamma, double dt) {
  int64_t np = n / 2;
  double lnL = coulomb_log(gamma, n);
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < np; ++p) {
    pair_geo g;
    pair_geometry(n, p, r, m, vr, vt, id, src, 1, lnL, &g);
    double beta = beta_of(g.tp, dt);
    if (!(g.wm > 0.0) || beta == 0.0) continue;
    int64_t a = g.a, b = g.b;

    double e1[3] = {g.w[0] / g.wm, g.w[1] / g.wm, g.w[2] / g.wm};
    double ax = fabs(g.w[0]), ay = fabs(g.w[1]), az = fabs(g.w[2]);
    double c[3];
    if (ax <= ay && ax <= az) { /* e1 x x-hat */
      c[0] = 0.0;
      c[1] = e1[2];
      c[2] = -e1[1];
    } else if (ay <= az) { /* e1 x y-hat */
      c[0] = -e1[2];
      c[1] = 0.0;
      c[2] = e1[0];
    } else { /* e1 x z-hat */
      c[0] = e1[1];
      c[1] = -e1[0];
      c[2] = 0.0;
    }
    double cn = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    double e2[3] = {c[0] / cn, c[1] / cn, c[2] / cn};
    double e3[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                    e1[0] * e2[1] - e1[1] * e2[0]};
    double psi2 = 2.0 * PI * g.u2;
    double cb = cos(beta), sb = sin(beta), cp = cos(psi2), sp = sin(psi2);
    double wn[3];
    for (int d = 0; d < 3; ++d) wn[d] = g.wm * (cb * e1[d] + sb * (cp * e2[d] + sp * e3[d]));

    double v1[3] = {vr[a], vt[a], 0.0};
    const double *v2 = g.v2;
    double ms = m[a] + m[b];
    double fa = m[a] / ms, fb = m[b] / ms;
    double vcm[3], n1[3], n2[3];
    for (int d = 0; d < 3; ++d) {
      vcm[d] = fa * v1[d] + fb * v2[d];
      n1[d] = vcm[d] + fb * wn[d];
      n2[d] = vcm[d] - fa * wn[d];
    }
    vr[a] = n1[0];
    vt[a] = hypot(n1[1], n1[2]);
    vr[b] = n2[0];
    vt[b] = hypot(n2[1], n2[2]);
  }
}

void ora_relax(int64_t n, const double *r, const double *m, double *vr, double *vt,
               const uint32_t *id, uint64_t seed, uint32_t step, double gamma, double dt) {
  const draws src = {seed, step, NULL};
  relax_d(n, r, m, vr, vt, id, &src, gamma, dt);
}

/* ------------------------------------------------------------------------- */
/* New orbits (Sec. 2.1 step 5).  Q(r) = 2E - 2Phi(r) - J^2/r^2; the paper
 * brackets each turning point between table radii by bisection, solves it
 * analytically inside the bracket, and draws the new radius with probability
 * dt/T = (dr/|v_r|)/integral by von Neumann rejection.  The endpoint
 * singularity of 1/|v_r| is removed by r = r_c + r_a sin s, s in (-pi/2,
 * pi/2), under which the density in s is g(s) = r_a cos s / sqrt(Q(r)),
 * finite at both ends: g(+-pi/2) = sqrt(2 r_a / |Q'(r_end)|) at a simple root.
 * The bound is F = bound_factor * max(g(-pi/2), g(pi/2)).  The table (r, Phi,
 * M) is frozen for the whole pass: the orbit is drawn in the old potential. */

/* Q at table index k; sentinels k = -1 (r = 0) and k = n (r = inf).  A star
 * sitting exactly at r = 0 takes the limit r -> 0 of Q(r): -inf when J != 0
 * (the J^2/r^2 term dominates, also against Phi = -inf from the star's own
 * m/r), else 2E - 2 Phi_k. */
static double q_at(int64_t n, const double *r, const double *phi, int64_t k, double E,
                   double J2) {
  if (k < 0) return -INFINITY;
  if (k >= n) return 2.0 * E;
  if (r[k] == 0.0) return (J2 > 0.0) ? -INFINITY : 2.0 * E - 2.0 * phi[k];
  return 2.0 * E - 2.0 * phi[k] - J2 / (r[k] * r[k]);
}

/* dQ/dr inside interval k. */
static double dq_in(const double *mcum, int64_t k, double x, double J2) {
  double grav = (k >= 0) ? -2.0 * mcum[k] / (x * x) : 0.0;
  return grav + 2.0 * J2 / (x * x * x);
}

/* One star's share of the pass's tallies. */
typedef struct {
  int32_t esc, capped, trials, violations;
  uint32_t fl;
  double m_e; /* m E of an escaper */
} star_tally;

static void orbit_d(int64_t n, const double *r, const double *phi, const double *mcum,
                    const double *ssuf, const double *m, double *vr, double *vt,
                    const uint32_t *id, const draws *src, int32_t trial_cap,
                    double bound_factor, double *r_new, double *E_out, double *J_out,
                    int64_t *kmin_out, int64_t *kmax_out, double *rmin_out,
                    double *rmax_out, int32_t *trials_out, uint32_t *flags_out,
                    ora_orbit_stats *st, const int64_t *only, int64_t count) {
  ora_orbit_stats s;
  memset(&s, 0, sizeof s);
  ksum eesc = {0.0, 0.0};

  /* every star, or only the listed ones (each star's orbit depends on the
   * table and its own state alone); each star's tallies are kept apart and
   * summed in star order after the loop, so the result does not depend on
   * whether the loop runs on one thread or many */
  const int64_t todo = only ? count : n;
  star_tally *tally = (star_tally *)calloc((size_t)(todo > 0 ? todo : 1), sizeof(star_tally));
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t q = 0; q < todo; ++q) {
    const int64_t i = only ? only[q] : q;
    star_tally *t = &tally[q];
    uint32_t fl = 0;
    double E = phi[i] + 0.5 * (vr[i] * vr[i] + vt[i] * vt[i]);
    double J = r[i] * vt[i];
    double J2 = J * J;
    if (E_out) E_out[i] = E;
    if (J_out) J_out[i] = J;
    if (!(E < 0.0)) { /* unbound (or not a number): leaves the cluster */
      r_new[i] = INFINITY;
      t->esc = 1;
      t->m_e = m[i] * E;
      fl |= ORA_ST_ESCAPER;
      if (E != E) fl |= ORA_ST_NONFINITE;
      t->fl = fl;
      if (flags_out) flags_out[i] = fl;
      if (kmin_out) kmin_out[i] = -2;
      if (kmax_out) kmax_out[i] = -2;
      if (rmin_out) rmin_out[i] = NAN;
      if (rmax_out) rmax_out[i] = NAN;
      if (trials_out) trials_out[i] = 0;
      continue;
    }

    /* Brackets by bisection.  Q at the star's own index is v_r^2 >= 0 (taken
     * as non-negative), Q(0+) < 0 and Q(inf) = 2E < 0, and Q changes sign
     * once on each side because M(r) r increases with r. */
    int64_t lo = -1, hi = i;
    while (hi - lo > 1) {
      int64_t mid = lo + (hi - lo) / 2;
      if (q_at(n, r, phi, mid, E, J2) < 0.0)
        lo = mid;
      else
        hi = mid;
    }
    int64_t kmin = lo;
    lo = i;
    hi = n;
    while (hi - lo > 1) {
      int64_t mid = lo + (hi - lo) / 2;
      if (q_at(n, r, phi, mid, E, J2) >= 0.0)
        lo = mid;
      else
        hi = mid;
    }
    int64_t kmax = lo;

    /* Roots inside the brackets: r^2 Q(r) = a r^2 + b r - J^2 with
     * a = 2 (E + S_k), b = 2 M_k; stable quadratic forms. */
    double rmin, rmax;
    if (J2 == 0.0) {
      rmin = 0.0;
    } else if (kmin < 0) {
      rmin = J / sqrt(2.0 * (E - phi[0]));
    } else {
      double a = 2.0 * (E + ssuf[kmin]);
      double b = 2.0 * mcum[kmin];
      double disc = b * b + 4.0 * a * J2;
      double sq = sqrt(disc > 0.0 ? disc : 0.0);
      double den = b + sq;
      rmin = (den > 0.0) ? 2.0 * J2 / den : r[kmin];
    }
    {
      double rl = (kmin >= 0) ? r[kmin] : 0.0, rh = r[kmin + 1];
      if (rmin < rl) rmin = rl;
      if (rmin > rh) rmin = rh;
    }
    {
      double a = 2.0 * (E + ssuf[kmax]);
      double b = 2.0 * mcum[kmax];
      double disc = b * b + 4.0 * a * J2;
      double sq = sqrt(disc > 0.0 ? disc : 0.0);
      double rh = (kmax + 1 < n) ? r[kmax + 1] : INFINITY;
      rmax = (a < 0.0) ? (b + sq) / (-2.0 * a) : rh;
      if (rmax < r[kmax]) rmax = r[kmax];
      if (rmax > rh) rmax = rh;
    }
    if (kmin_out) kmin_out[i] = kmin;
    if (kmax_out) kmax_out[i] = kmax;
    if (rmin_out) rmin_out[i] = rmin;
    if (rmax_out) rmax_out[i] = rmax;

    /* Rejection sampling in s. */
    double rc = 0.5 * (rmax + rmin), ra = 0.5 * (rmax - rmin);
    double r0 = rmin;
    int32_t ntr = 0;
    if (ra > 0.0) {
      double glo = 0.0, ghi;
      if (J2 != 0.0) glo = sqrt(2.0 * ra / fabs(dq_in(mcum, kmin, rmin, J2)));
      ghi = sqrt(2.0 * ra / fabs(dq_in(mcum, kmax, rmax, J2)));
      double F = bound_factor * (glo > ghi ? glo : ghi);
      if (F > 0.0 && F < INFINITY) {
        int accepted = 0;
        for (int32_t j = 0; j < trial_cap; ++j) {
          uint32_t w[4];
          star_draw(src, id, i, ORA_P_ORBIT, (uint32_t)j, 1, w);
          double X = ora_u01(w[1], w[0]);
          double X2 = ora_u01(w[3], w[2]);
          double s0 = PI * (X - 0.5);
          r0 = rc + ra * sin(s0);
          ++ntr;
          int64_t k0 = interval_of(r, kmin, kmax, r0);
          double q0 = 2.0 * E - 2.0 * phi_in(phi, mcum, ssuf, k0, r0) - J2 / (r0 * r0);
          if (!(q0 > 0.0)) continue;
          double g0 = ra * cos(s0) / sqrt(q0);
          if (g0 > F) {
            t->violations++;
            fl |= ORA_ST_BOUND;
          }
          if (F * X2 < g0) {
            accepted = 1;
            break;
          }
        }
        if (!accepted) {
          t->capped = 1;
          fl |= ORA_ST_TRIAL_CAP;
        }
      } else {
        r0 = rc;
        fl |= ORA_ST_NUMERIC;
      }
    }
    t->trials = ntr;
    if (trials_out) trials_out[i] = ntr;

    /* New state: J conserved, E conserved in the old potential, random sign
     * of v_r. */
    double rn = r0 + 0.0;
    int64_t kn = interval_of(r, kmin, kmax, rn);
    double qn = 2.0 * E - 2.0 * phi_in(phi, mcum, ssuf, kn, rn) - (J2 == 0.0 ? 0.0 : J2 / (rn * rn));
    uint32_t w[4];
    star_draw(src, id, i, ORA_P_SIGN, 0u, 1, w);
    double vmag = sqrt(qn > 0.0 ? qn : 0.0);
    r_new[i] = rn;
    vr[i] = (w[0] >> 31) ? -vmag : vmag;
    vt[i] = (J2 == 0.0) ? 0.0 : J / rn;
    if (!isfinite(rn) || !isfinite(vr[i]) || !isfinite(vt[i])) fl |= ORA_ST_NONFINITE;
    t->fl = fl;
    if (flags_out) flags_out[i] = fl;
  }
  for (int64_t q = 0; q < todo; ++q) {
    const star_tally *t = &tally[q];
    if (t->esc) {
      s.n_esc++;
      kadd(&eesc, t->m_e);
    }
    s.violations += t->violations;
    s.capped += t->capped;
    s.trials += t->trials;
    s.status |= t->fl;
  }
  free(tally);
  s.e_esc = kval(&eesc);
  if (st) *st = s;
}

void ora_orbit(int64_t n, const double *r, const double *phi, const double *mcum,
               const double *ssuf, const double *m, double *vr, double *vt, const uint32_t *id,
               uint64_t seed, uint32_t step, int32_t trial_cap, double bound_factor,
               double *r_new, double *E_out, double *J_out, int64_t *kmin_out,
               int64_t *kmax_out, double *rmin_out, double *rmax_out, int32_t *trials_out,
               uint32_t *flags_out, ora_orbit_stats *st) {
  const draws src = {seed, step, NULL};
  orbit_d(n, r, phi, mcum, ssuf, m, vr, vt, id, &src, trial_cap, bound_factor, r_new, E_out,
          J_out, kmin_out, kmax_out, rmin_out, rmax_out, trials_out, flags_out, st, NULL, 0);
}

void ora_orbit_subset(int64_t n, const double *r, const double *phi, const double *mcum,
                      const double *ssuf, const double *m, double *vr, double *vt,
                      const uint32_t *id, uint64_t seed, uint32_t step, int32_t trial_cap,
                      double bound_factor, int64_t count, const int64_t *idx, double *r_new) {
  const draws src = {seed, step, NULL};
  orbit_d(n, r, phi, mcum, ssuf, m, vr, vt, id, &src, trial_cap, bound_factor, r_new, NULL,
          NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, idx, count);
}

/* ------------------------------------------------------------------------- */
void ora_step(int64_t n, double *r, double *vr, double *vt, double *m, uint32_t *id,
              double *phi, double *mcum, const ora_params *p, ora_step_out *out) {
  ora_step_ex(n, r, vr, vt, m, id, phi, mcum, p, out, NULL, NULL);
}

void ora_step_ex(int64_t n, double *r, double *vr, double *vt, double *m, uint32_t *id,
                 double *phi, double *mcum, const ora_params *p, ora_step_out *out,
                 double *moves, uint32_t *lfsr) {
  const draws src = {p->seed, p->step, lfsr};
  size_t nn = (size_t)(n > 0 ? n : 1);
  uint32_t status = 0;
  double *ssuf = (double *)malloc(nn * sizeof(double));
  ora_potential(n, r, m, phi, mcum, ssuf);

  int64_t np = n / 2;
  double *w = (double *)malloc((np > 0 ? (size_t)np : 1) * sizeof(double));
  double *tp = (double *)malloc((np > 0 ? (size_t)np : 1) * sizeof(double));
  pair_terms_d(n, r, m, vr, vt, id, &src, p->gamma, w, tp, NULL);
  double dt = (p->dt_fixed > 0.0) ? p->dt_fixed : ora_solve_dt(np, w, tp, p->target, &status);
  free(w);
  free(tp);

  relax_d(n, r, m, vr, vt, id, &src, p->gamma, dt);

  double *rn = (double *)malloc(nn * sizeof(double));
  ora_orbit_stats st;
  orbit_d(n, r, phi, mcum, ssuf, m, vr, vt, id, &src, p->trial_cap, p->bound_factor, rn,
          NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, &st, NULL, 0);
  status |= st.status;

  /* The old potential at each star's old and new radius (for the energy
   * correction of the next potential). */
  double *phi_rn = NULL;
  if (moves) {
    phi_rn = (double *)malloc(nn * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
      phi_rn[i] = (rn[i] < INFINITY) ? ora_phi_at(n, r, phi, mcum, ssuf, rn[i]) : NAN;
  }

  int64_t *perm = (int64_t *)malloc(nn * sizeof(int64_t));
  ora_sort_perm(n, rn, perm);
  double *t_r = (double *)malloc(nn * sizeof(double));
  double *t_vr = (double *)malloc(nn * sizeof(double));
  double *t_vt = (double *)malloc(nn * sizeof(double));
  double *t_m = (double *)malloc(nn * sizeof(double));
  uint32_t *t_id = (uint32_t *)malloc(nn * sizeof(uint32_t));
  uint32_t *t_lfsr = lfsr ? (uint32_t *)malloc(4 * nn * sizeof(uint32_t)) : NULL;
  int64_t kept = 0;
  for (int64_t q = 0; q < n; ++q) {
    int64_t o = perm[q];
    t_r[q] = rn[o];
    t_vr[q] = vr[o];
    t_vt[q] = vt[o];
    t_m[q] = m[o];
    t_id[q] = id[o];
    if (lfsr) memcpy(t_lfsr + 4 * q, lfsr + 4 * o, 4 * sizeof(uint32_t));
    if (rn[o] < INFINITY) {
      ++kept;
      if (moves) {
        moves[3 * q] = r[o];
        moves[3 * q + 1] = phi[o];
        moves[3 * q + 2] = phi_rn[o];
      }
    }
  }
  free(phi_rn);
  memcpy(r, t_r, nn * sizeof(double));
  memcpy(vr, t_vr, nn * sizeof(double));
  memcpy(vt, t_vt, nn * sizeof(double));
  memcpy(m, t_m, nn * sizeof(double));
  memcpy(id, t_id, nn * sizeof(uint32_t));
  if (lfsr) memcpy(lfsr, t_lfsr, 4 * nn * sizeof(uint32_t));
  free(t_lfsr);
  free(t_r);
  free(t_vr);
  free(t_vt);
  free(t_m);
  free(t_id);
  free(perm);
  free(rn);
  free(ssuf);

  if (out) {
    out->dt = dt;
    out->n_after = kept;
    out->orbit = st;
    out->status = status;
  }
}

/* ------------------------------------------------------------------------- */
/* Energy correction (Sec. 2.1 item 6).  A star's new orbit is drawn in the
 * potential of the old positions, Phi_old; once every star has moved the
 * potential is Phi_new.  Taking the potential to change linearly in time over
 * the step, the work it does on a star that goes from r_old to r_new is the
 * mean of the change dPhi = Phi_new - Phi_old at the two ends, so the star's
 * energy in the new potential should be E_old + (dPhi(r_old) + dPhi(r_new))/2.
 * As drawn it is E_old + dPhi(r_new) (its kinetic energy was fixed by
 * Phi_old(r_new)), so the kinetic energy per unit mass changes by
 *   dT = (dPhi(r_old) - dPhi(r_new)) / 2,
 * applied by scaling vr and vt by one factor (vr/vt unchanged).  A star whose
 * kinetic energy would not stay positive, or that has none to scale, keeps
 * its velocities and is counted.  Phi_new(r_old) is the defining sum over the
 * new state, -sum_j m_j / max(r_old, r_j); Phi_new(r_new) is phi. */
int64_t ora_energy_correction(int64_t n, const double *r, const double *m, double *vr,
                              double *vt, const double *phi, const double *moves) {
  int64_t skipped = 0;
  for (int64_t q = 0; q < n; ++q) {
    const double r_old = moves[3 * q], phi_old_at_old = moves[3 * q + 1];
    const double phi_old_at_new = moves[3 * q + 2];
    ksum s = {0.0, 0.0};
    for (int64_t j = 0; j < n; ++j) kadd(&s, m[j] / (r_old > r[j] ? r_old : r[j]));
    const double phi_new_at_old = -kval(&s);
    const double dT = 0.5 * ((phi_new_at_old - phi_old_at_old) - (phi[q] - phi_old_at_new));
    if (dT == 0.0) continue;
    const double v2 = vr[q] * vr[q] + vt[q] * vt[q];
    if (!(v2 > 0.0) || !(v2 + 2.0 * dT > 0.0)) {
      ++skipped;
      continue;
    }
    const double f = sqrt(1.0 + 2.0 * dT / v2);
    vr[q] *= f;
    vt[q] *= f;
  }
  return skipped;
}

/* ------------------------------------------------------------------------- */
void ora_diagnostics(int64_t n, const double *r, const double *vr, const double *vt,
                     const double *m, const double *phi, const double *mcum, double *out) {
  ksum T = {0.0, 0.0}, W = {0.0, 0.0};
  for (int64_t k = 0; k < n; ++k) {
    kadd(&T, 0.5 * m[k] * (vr[k] * vr[k] + vt[k] * vt[k]));
    kadd(&W, 0.5 * m[k] * phi[k]);
  }
  double t = kval(&T), wv = kval(&W);
  double M = (n > 0) ? mcum[n - 1] : 0.0;
  out[0] = t;
  out[1] = wv;
  out[2] = t + wv;
  out[3] = (wv != 0.0) ? 2.0 * t / fabs(wv) : 0.0;
  out[4] = M;
  const double fr[4] = {0.01, 0.1, 0.5, 0.9};
  for (int f = 0; f < 4; ++f) {
    double x = NAN;
    for (int64_t k = 0; k < n; ++k) {
      if (mcum[k] >= fr[f] * M) {
        x = r[k];
        break;
      }
    }
    out[5 + f] = x;
  }
  /* Core (the paper's core-collapse runs, after Casertano & Hut 1985): the
   * density around star i from its radial neighbours -- the 7 consecutive
   * stars a..a+6 that hold i near their middle, the mass of the 5 strictly
   * inside over the shell volume between r_a and r_(a+6) -- then the core
   * density sum rho_i^2 / sum rho_i and the density-weighted radius
   * sum rho_i r_i / sum rho_i.  A window of zero volume is left out. */
  ksum S1 = {0.0, 0.0}, S2 = {0.0, 0.0}, SR = {0.0, 0.0};
  int64_t used = 0;
  for (int64_t i = 0; n >= 7 && i < n; ++i) {
    int64_t a = i - 3;
    if (a < 0) a = 0;
    if (a > n - 7) a = n - 7;
    const double lo = r[a], hi = r[a + 6];
    const double vol = (4.0 * PI / 3.0) * (hi - lo) * (hi * hi + hi * lo + lo * lo);
    if (!(vol > 0.0)) continue;
    double inner = 0.0;
    for (int64_t k = a + 1; k <= a + 5; ++k) inner += m[k];
    const double rho = inner / vol;
    kadd(&S1, rho);
    kadd(&S2, rho * rho);
    kadd(&SR, rho * r[i]);
    ++used;
  }
  const double s1 = kval(&S1);
  out[9] = (used > 0 && s1 > 0.0) ? kval(&SR) / s1 : NAN;
  out[10] = (used > 0 && s1 > 0.0) ? kval(&S2) / s1 : NAN;
}

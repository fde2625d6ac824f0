// init.hip -- initial models (arXiv:1206.5878, Sec. 2.1 opening paragraph:
// sample mass, radius and the radial/transverse velocity from the
// distribution function, keep only |r|, vr, vt, start sorted by radius).
//
// Plummer.  Star i draws from Philox counter (i, 0, purpose, trial):
//   r = (X1^(-2/3) - 1)^(-1/2), written sqrt(y / (1 - y)) with y = X1^(2/3) and
//       1 - y = -expm1((2/3) ln X1) for full precision in the tail;
//   q by rejection on q^2 (1 - q^2)^(7/2) < 0.1 X5, v = q sqrt(2) (1+r^2)^(-1/4);
//   cos(theta) = 2 X6 - 1, vr = v cos(theta), vt = v sin(theta);
//   Henon units: r * 3pi/16, v * sqrt(16/(3pi)).
// Masses: 1/n, or a broken power law (slopes -1.3 on [0.1,0.5] and -2.3 on
// [0.5,100], continuous at 0.5) by inverse CDF per segment, divided by their
// total at the final gather.
//
// King (1966), central potential W0.  In units G = sigma = r_K = 1 the
// dimensionless potential obeys W'' + 2W'/r = -9 rho(W)/rho(W0) with
// rho(W) = e^W erf(sqrt W) - sqrt(4W/pi) (1 + 2W/3), W(0) = W0, W'(0) = 0, and
// M(r) = -r^2 W'.  One thread per cluster integrates (W, U = r^2 W') by RK4
// in ln r from r = 1e-4 (series start) until W crosses 0 (the tidal radius),
// tabulating (r, W, M).  A star takes r from the inverse of M(r) (linear
// between nodes), its speed by rejection on v^2 (e^(W - v^2/2) - 1),
// v < sqrt(2W), an isotropic direction, and the model is scaled to Henon
// units (G = M = 1, E = -1/4) with E = W_pot / 2 (virial equilibrium),
// W_pot = -integral M dM / r by the trapezoid rule over the nodes.
//
// The records go through the radial sort.
#include <type_traits>

#include "cmc_internal.hpp"

namespace cmc {
namespace {

constexpr int NT = kBlock;
constexpr double kKingR0 = 1e-4;    // series start of the King integration
constexpr double kKingDlnr = 0.005;  // RK4 step in ln r

// One thread per cluster.
template <class Ctx>
__global__ void k_clear_scalars(Ctx ctx) {
  const ClusterArgs &A = ctx.args();
  cmc_scalars *sc = A.s.sc;
  sc->n = A.n_init;
  sc->dt = 0.0;
  sc->status = 0u;
  sc->dt_iters = 0u;
  sc->n_esc = 0;
  sc->trials = 0;
  sc->violations = 0;
  sc->capped = 0;
  sc->e_esc = 0.0;
  sc->mass_norm = 1.0;
  sc->step = 0;
  sc->corr_n = 0;
  sc->corr_skipped = 0;
  for (int q = 0; q < 4; ++q) sc->reserved[q] = 0;
}

// King density up to a constant; the series for small W avoids the
// cancellation of the closed form.
__device__ double king_rho(double W) {
  if (!(W > 0.0)) return 0.0;
  if (W < 0.1) {
    // e^W erf(sqrt W) = (2/sqrt pi) sqrt W sum_n (2W)^n / (2n+1)!!
    double term = 4.0 * W * W / 15.0, sum = 0.0;
    for (int k = 2; k < 12; ++k) {
      sum += term;
      term *= 2.0 * W / (2.0 * k + 3.0);
    }
    return (2.0 / sqrt(kPi)) * sqrt(W) * sum;
  }
  return exp(W) * erf(sqrt(W)) - sqrt(4.0 * W / kPi) * (1.0 + 2.0 * W / 3.0);
}

// Table layout in w.king: r[kKingNodes], W[kKingNodes], M[kKingNodes], then
// nodes, r_t, M_t, W_pot.
__device__ __forceinline__ void king_deriv(double t, double W, double U, double rho0,
                                           double &dW, double &dU) {
  const double r = exp(t);
  dW = U / r;                                  // dW/dln r = r W' = U / r
  dU = -9.0 * r * r * r * king_rho(W) / rho0;  // dU/dln r = r dU/dr
}

template <class Ctx>
__global__ void k_king_profile(Ctx ctx) {
  const ClusterArgs &A = ctx.args();
  if (A.model != CMC_MODEL_KING) return;
  double *kr = A.w.king, *kW = kr + kKingNodes, *kM = kW + kKingNodes, *tail = kM + kKingNodes;
  const double W0 = A.w0;
  const double rho0 = king_rho(W0);
  const double a = (exp(W0) * erf(sqrt(W0)) - sqrt(4.0 * W0 / kPi)) / rho0;  // rho'/rho at W0
  double r = kKingR0;
  double W = W0 - 1.5 * r * r + 0.675 * a * r * r * r * r;
  double U = -3.0 * r * r * r + 2.7 * a * r * r * r * r * r;
  double t = log(r);
  int k = 0;
  kr[0] = r;
  kW[0] = W;
  kM[0] = -U;
  double rt = r, Mt = -U;
  while (k + 2 < kKingNodes) {
    double d1W, d1U, d2W, d2U, d3W, d3U, d4W, d4U;
    const double h = kKingDlnr;
    king_deriv(t, W, U, rho0, d1W, d1U);
    king_deriv(t + 0.5 * h, W + 0.5 * h * d1W, U + 0.5 * h * d1U, rho0, d2W, d2U);
    king_deriv(t + 0.5 * h, W + 0.5 * h * d2W, U + 0.5 * h * d2U, rho0, d3W, d3U);
    king_deriv(t + h, W + h * d3W, U + h * d3U, rho0, d4W, d4U);
    const double Wn = W + (h / 6.0) * (d1W + 2.0 * d2W + 2.0 * d3W + d4W);
    const double Un = U + (h / 6.0) * (d1U + 2.0 * d2U + 2.0 * d3U + d4U);
    const double tn = t + h;
    if (!(Wn > 0.0)) {  // the tidal radius lies in this step: interpolate
      const double f = W / (W - Wn);
      rt = exp(t + f * h);
      Mt = -(U + f * (Un - U));
      break;
    }
    W = Wn;
    U = Un;
    t = tn;
    ++k;
    kr[k] = exp(t);
    kW[k] = W;
    kM[k] = -U;
    rt = kr[k];
    Mt = -U;
  }
  ++k;  // the tidal node
  kr[k] = rt;
  kW[k] = 0.0;
  kM[k] = Mt;
  // W_pot = -integral M dM / r over the nodes (trapezoid in M)
  double wpot = 0.0;
  for (int q = 0; q < k; ++q)
    wpot -= 0.5 * (kM[q] / kr[q] + kM[q + 1] / kr[q + 1]) * (kM[q + 1] - kM[q]);
  tail[0] = static_cast<double>(k + 1);
  tail[1] = rt;
  tail[2] = Mt;
  tail[3] = wpot;
}

template <class Ctx>
__global__ __launch_bounds__(NT) void k_init(Ctx ctx) {
  __shared__ double sh[NT / 64];
  const ClusterArgs &A = ctx.args();
  const int64_t n = A.n_init;
  const uint64_t seed = A.seed;
  const int king = A.model == CMC_MODEL_KING;
  const int mass_spectrum = A.mass_spectrum;
  WideRec *__restrict__ stage = static_cast<WideRec *>(A.w.stage);
  uint64_t *__restrict__ keys = A.w.keys[0];
  const int64_t blk = ctx.block();
  const int64_t i = blk * NT + threadIdx.x;
  double mraw = 0.0;
  if (i < n) {
    const uint32_t ii = static_cast<uint32_t>(i);
    U4 w = philox(ii, 0u, kInitPos, 0u, seed);
    const double x1 = u01(w.y, w.x), x6 = u01(w.w, w.z);
    double rr, vv;
    if (king) {
      const double *kr = A.w.king, *kW = kr + kKingNodes, *kM = kW + kKingNodes;
      const double *tail = kM + kKingNodes;
      const int nodes = static_cast<int>(tail[0]);
      const double Mt = tail[2], wpot = tail[3];
      // radius: inverse of M(r), linear between nodes; r^3 law inside the first
      const double Mx = x1 * Mt;
      double Wr;
      if (Mx < kM[0]) {
        rr = cbrt(Mx / 3.0);
        Wr = A.w0 - 1.5 * rr * rr;
      } else {
        int lo = 0, hi = nodes - 1;  // kM[lo] <= Mx < kM[hi]
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (kM[mid] <= Mx) lo = mid; else hi = mid;
        }
        const double f = (Mx - kM[lo]) / (kM[hi] - kM[lo]);
        rr = kr[lo] + f * (kr[hi] - kr[lo]);
        Wr = kW[lo] + f * (kW[hi] - kW[lo]);
      }
      // speed: v^2 (e^(W - v^2/2) - 1) on v < sqrt(2W), bounded by max v^2 e^(W - v^2/2)
      double v = 0.0;
      if (Wr > 0.0) {
#pragma clang fp contract(off)
        const double vmax = sqrt(2.0 * Wr);
        const double bound = Wr >= 1.0 ? 2.0 * exp(Wr - 1.0) : 2.0 * Wr;
        for (uint32_t j = 0; j < 1000000u; ++j) {
          w = philox(ii, 0u, kInitSpeed, j, seed);
          v = vmax * u01(w.y, w.x);
          const double x5 = u01(w.w, w.z);
          if (x5 * bound < v * v * expm1(Wr - 0.5 * v * v)) break;
        }
      }
      // Henon units
      const double s = -4.0 * (0.5 * wpot) / (Mt * Mt);
      rr = rr * s;
      vv = v / sqrt(Mt * s);
    } else {
      const double lx = (2.0 / 3.0) * log(x1);
      const double r0 = sqrt(exp(lx) / -expm1(lx));
      double q = 0.0;
      {
        // the comparison that decides a trial is evaluated without contraction
        // so it rounds like the plain IEEE expression
#pragma clang fp contract(off)
        for (uint32_t j = 0; j < 1000000u; ++j) {
          w = philox(ii, 0u, kInitSpeed, j, seed);
          q = u01(w.y, w.x);
          const double x5 = u01(w.w, w.z);
          const double t = 1.0 - q * q;
          const double g = q * q * (t * t * t) * sqrt(t);
          if (0.1 * x5 < g) break;
        }
      }
      const double v = q * sqrt(2.0) * pow(1.0 + r0 * r0, -0.25);
      rr = r0 * (3.0 * kPi / 16.0);
      vv = v * sqrt(16.0 / (3.0 * kPi));
    }
    const double c = 2.0 * x6 - 1.0;
    const double sn = sqrt((1.0 - c) * (1.0 + c));
    WideRec rec;
    rec.r = rr;
    rec.vr = vv * c;
    rec.vt = vv * sn;
    if (mass_spectrum) {
      w = philox(ii, 0u, kInitMass, 0u, seed);
      const double us = u01(w.y, w.x), um = u01(w.w, w.z);
      const double ia = (pow(0.1, -0.3) - pow(0.5, -0.3)) / 0.3;
      const double ib = 0.5 * (pow(0.5, -1.3) - pow(100.0, -1.3)) / 1.3;
      const double f1 = ia / (ia + ib);
      if (us < f1) {
        const double lo = pow(0.1, -0.3), hi = pow(0.5, -0.3);
        mraw = pow(lo - um * (lo - hi), -1.0 / 0.3);
      } else {
        const double lo = pow(0.5, -1.3), hi = pow(100.0, -1.3);
        mraw = pow(lo - um * (lo - hi), -1.0 / 1.3);
      }
    } else {
      mraw = 1.0 / static_cast<double>(n);
    }
    rec.m = mraw;
    rec.id = ii;
    rec.pad = 0u;
    stage[i] = rec;
    keys[i] = __builtin_bit_cast(uint64_t, rec.r + 0.0);
  }
  if (!mass_spectrum) return;
  // total raw mass: block partials, summed in block order by k_mass_total
  const double bs = block_sum<NT>(mraw, sh);
  if (threadIdx.x == 0) A.w.red_part[blk] = bs;
}

constexpr int FT = 1024;

// One block per cluster.
template <class Ctx>
__global__ __launch_bounds__(FT) void k_mass_total(Ctx ctx) {
  __shared__ double sh[FT / 64];
  const ClusterArgs &A = ctx.args();
  if (!A.mass_spectrum) return;
  const int64_t nblocks = cdiv(A.n_init > 0 ? A.n_init : 1, NT);
  double t = 0.0;
  for (int64_t b = threadIdx.x; b < nblocks; b += FT) t += A.w.red_part[b];
  t = block_sum<FT>(t, sh);
  if (threadIdx.x == 0) A.s.sc->mass_norm = t;
}

}  // namespace

hipError_t launch_init(const Target &t, bool m_f32, hipStream_t st) {
  hipError_t e = dispatch(t, [&](const auto &l) {
    k_clear_scalars<<<l.grid(kShOne), 1, 0, st>>>(l.ctx(kShOne));
    k_king_profile<<<l.grid(kShOne), 1, 0, st>>>(l.ctx(kShOne));
    k_init<<<l.grid(kShStar), NT, 0, st>>>(l.ctx(kShStar));
    k_mass_total<<<l.grid(kShOne), FT, 0, st>>>(l.ctx(kShOne));
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  return launch_sort_stage(t, m_f32, true, false, false, false, st);
}

}  // namespace cmc

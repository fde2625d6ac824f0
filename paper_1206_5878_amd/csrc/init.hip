// init.hip -- initial Plummer model (arXiv:1206.5878, Sec. 2.1 opening
// paragraph: sample mass, radius and the radial/transverse velocity from the
// distribution function, keep only |r|, vr, vt, start sorted by radius).
// Star i draws from Philox counter (i, 0, purpose, trial):
//   r = (X1^(-2/3) - 1)^(-1/2), written sqrt(y / (1 - y)) with y = X1^(2/3) and
//       1 - y = -expm1((2/3) ln X1) for full precision in the tail;
//   q by rejection on q^2 (1 - q^2)^(7/2) < 0.1 X5, v = q sqrt(2) (1+r^2)^(-1/4);
//   cos(theta) = 2 X6 - 1, vr = v cos(theta), vt = v sin(theta);
//   Henon units: r * 3pi/16, v * sqrt(16/(3pi)).
// Masses: 1/n, or a broken power law (slopes -1.3 on [0.1,0.5] and -2.3 on
// [0.5,100], continuous at 0.5) by inverse CDF per segment, divided by their
// total at the final gather.  The records go through the radial sort.
#include "cmc_internal.hpp"

namespace cmc {
namespace {

constexpr int NT = kBlock;

__global__ void k_clear_scalars(cmc_scalars *__restrict__ sc, int64_t n) {
  sc->n = n;
  sc->dt = 0.0;
  sc->status = 0u;
  sc->dt_iters = 0u;
  sc->n_esc = 0;
  sc->trials = 0;
  sc->violations = 0;
  sc->capped = 0;
  sc->e_esc = 0.0;
  sc->mass_norm = 1.0;
  for (int q = 0; q < 7; ++q) sc->reserved[q] = 0;
}

__global__ __launch_bounds__(NT) void k_plummer(int64_t n, uint64_t seed, int mass_spectrum,
                                                StageRec *__restrict__ stage,
                                                uint64_t *__restrict__ keys,
                                                double *__restrict__ part) {
  __shared__ double sh[NT / 64];
  const int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
  double mraw = 0.0;
  if (i < n) {
    const uint32_t ii = static_cast<uint32_t>(i);
    U4 w = philox(ii, 0u, kInitPos, 0u, seed);
    const double x1 = u01(w.y, w.x), x6 = u01(w.w, w.z);
    const double lx = (2.0 / 3.0) * log(x1);
    const double rr = sqrt(exp(lx) / -expm1(lx));
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
    const double v = q * sqrt(2.0) * pow(1.0 + rr * rr, -0.25);
    const double c = 2.0 * x6 - 1.0;
    const double s = sqrt((1.0 - c) * (1.0 + c));
    const double vs = v * sqrt(16.0 / (3.0 * kPi));
    StageRec rec;
    rec.r = rr * (3.0 * kPi / 16.0);
    rec.vr = vs * c;
    rec.vt = vs * s;
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
  if (threadIdx.x == 0) part[blockIdx.x] = bs;
}

constexpr int FT = 1024;

__global__ __launch_bounds__(FT) void k_mass_total(const double *__restrict__ part,
                                                   int64_t nblocks, cmc_scalars *__restrict__ sc) {
  __shared__ double sh[FT / 64];
  double t = 0.0;
  for (int64_t b = threadIdx.x; b < nblocks; b += FT) t += part[b];
  t = block_sum<FT>(t, sh);
  if (threadIdx.x == 0) sc->mass_norm = t;
}

}  // namespace

hipError_t launch_init_plummer(const cmc_state &s, const Workspace &w, int64_t n,
                               uint64_t seed, int mass_spectrum, hipStream_t st) {
  k_clear_scalars<<<1, 1, 0, st>>>(s.sc, n);
  const unsigned nb = static_cast<unsigned>(cdiv(n > 0 ? n : 1, NT));
  k_plummer<<<nb, NT, 0, st>>>(n, seed, mass_spectrum, w.stage, w.keys[0], w.red_part);
  if (mass_spectrum) k_mass_total<<<1, FT, 0, st>>>(w.red_part, nb, s.sc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_sort_stage(s, w, mass_spectrum != 0, st);
}

}  // namespace cmc

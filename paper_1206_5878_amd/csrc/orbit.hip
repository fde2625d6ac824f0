// orbit.hip -- new orbits (arXiv:1206.5878, Sec. 2.1 step 5).  One thread per
// star: E = Phi_i + v^2/2 and J = r_i vt_i; the turning points are bracketed
// between table radii by the sign of Q_k = 2E - 2Phi_k - J^2/r_k^2 (negative,
// positive, negative over k), solved in the bracket from
// r^2 Q = 2(E + S_k) r^2 + 2 M_k r - J^2; the new radius is drawn with density
// ~ 1/|v_r| by rejection in r = r_c + r_a sin s, where the density in s,
// g(s) = r_a cos s / sqrt(Q), is finite at both turning points.  The table
// is read-only for the whole pass (old potential).
//
// Searches.  Each of the three lookups -- the lower bracket, the upper
// bracket, the interval of a trial radius -- is "the last index k where a
// predicate monotone in k holds".  It descends the sampled levels of the
// table (level L = every 8^L-th (r, Phi)): at every level it loads the 8
// children of the current sample, one aligned cache line, and counts how many
// satisfy the predicate.  The brackets and intervals are unique, so this
// finds the index a bisection over the whole table finds.
#include "cmc_internal.hpp"

namespace cmc {
namespace {

constexpr int NT = kBlock;

// Q_k < 0 as (2E - 2Phi_k) r_k^2 < J^2 (r_k > 0): no division in the descent.
struct QNeg {
  double twoE, J2;
  int64_t below;  // only indices < below can hold
  __device__ bool operator()(int64_t k, const RPhi &e) const {
    return k < below && (twoE - 2.0 * e.phi) * (e.r * e.r) < J2;
  }
};
// Q_k >= 0 or k <= upto.
struct QNonNeg {
  double twoE, J2;
  int64_t upto;
  __device__ bool operator()(int64_t k, const RPhi &e) const {
    return k <= upto || (twoE - 2.0 * e.phi) * (e.r * e.r) >= J2;
  }
};
// k <= klo, or k <= khi and r_k <= x.
struct RBelow {
  double x;
  int64_t klo, khi;
  __device__ bool operator()(int64_t k, const RPhi &e) const {
    return k <= klo || (k <= khi && e.r <= x);
  }
};

// Last k in [0, n-1] with pred(k) true (-1 if none); pred must be monotone
// (true ... true false ... false).
template <class Pred>
__device__ __forceinline__ int64_t last_true(const Levels &lv, int64_t n, const Pred &pred) {
  int L = lv.nlev - 1;
  int64_t stride = int64_t(1) << (3 * L);
  int64_t s = -1;
  {
    const int64_t cnt = (n + stride - 1) / stride;  // <= 8
    int c = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (q < cnt && pred(q * stride, lv.lev[L][q])) c = q + 1;
    s = c - 1;
  }
  if (s < 0) return -1;
  for (--L; L >= 0; --L) {
    stride >>= 3;
    const int64_t cnt = (n + stride - 1) / stride;
    const int64_t base = s * 8;  // child 0 is sample s itself: known true
    const RPhi *blk = lv.lev[L] + base;
    int c = 0;
    RPhi e[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) e[q] = (base + 1 + q < cnt) ? blk[1 + q] : RPhi{0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 7; ++q)
      if (base + 1 + q < cnt && pred((base + 1 + q) * stride, e[q])) c = q + 1;
    s = base + c;
  }
  return s;
}

// Potential inside interval k from the defining sum: -(M_k / x + S_k); flat
// at Phi_0 inside the innermost star.
__device__ __forceinline__ double phi_in(const Levels &lv, const MS *__restrict__ ms, int64_t k,
                                         double x) {
  if (k < 0) return lv.lev[0][0].phi;
  const MS t = ms[k];
  return -(t.M / x + t.S);
}

__device__ __forceinline__ double dq_in(const MS *__restrict__ ms, int64_t k, double x,
                                        double J2) {
  const double grav = (k >= 0) ? -2.0 * ms[k].M / (x * x) : 0.0;
  return grav + 2.0 * J2 / (x * x * x);
}

template <typename MT, bool TO_STAGE>
__global__ __launch_bounds__(NT) void k_orbit(
    Levels lv, const MS *__restrict__ ms, const MT *__restrict__ m, double *__restrict__ vr,
    double *__restrict__ vt, const uint32_t *__restrict__ id, double *__restrict__ r_new,
    StageRec *__restrict__ stage, uint64_t *__restrict__ keys, cmc_scalars *__restrict__ sc,
    double *__restrict__ part, uint64_t seed, uint32_t step, int32_t trial_cap,
    double bound_factor) {
  __shared__ double shd[NT / 64];
  const int64_t n = sc->n;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
  double c_esc = 0.0, c_tr = 0.0, c_viol = 0.0, c_cap = 0.0, e_esc = 0.0;
  uint32_t fl = 0;
  const RPhi *tab = lv.lev[0];

  if (i < n) {
    const RPhi me = tab[i];
    const double vri = vr[i], vti = vt[i], ri = me.r;
    const double E = me.phi + 0.5 * (vri * vri + vti * vti);
    const double J = ri * vti;
    const double J2 = J * J;
    const uint32_t sid = id[i];
    double rn = kInf, vrn = vri, vtn = vti;
    if (!(E < 0.0)) {
      c_esc = 1.0;
      e_esc = load_mass(m, i) * E;
      fl |= CMC_ST_ESCAPER;
      if (E != E) fl |= CMC_ST_NONFINITE;
    } else {
      const int64_t kmin = last_true(lv, n, QNeg{2.0 * E, J2, i});
      const int64_t kmax = last_true(lv, n, QNonNeg{2.0 * E, J2, i});

      // roots inside the brackets
      double rmin, rmax;
      if (J2 == 0.0) {
        rmin = 0.0;
      } else if (kmin < 0) {
        rmin = J / sqrt(2.0 * (E - tab[0].phi));
      } else {
        const MS t = ms[kmin];
        const double a = 2.0 * (E + t.S);
        const double b = 2.0 * t.M;
        const double disc = b * b + 4.0 * a * J2;
        const double den = b + sqrt(disc > 0.0 ? disc : 0.0);
        rmin = den > 0.0 ? 2.0 * J2 / den : tab[kmin].r;
      }
      {
        const double rl = kmin >= 0 ? tab[kmin].r : 0.0, rh = tab[kmin + 1].r;
        rmin = rmin < rl ? rl : (rmin > rh ? rh : rmin);
      }
      {
        const MS t = ms[kmax];
        const double a = 2.0 * (E + t.S);
        const double b = 2.0 * t.M;
        const double disc = b * b + 4.0 * a * J2;
        const double sq = sqrt(disc > 0.0 ? disc : 0.0);
        const double rl = tab[kmax].r;
        const double rh = (kmax + 1 < n) ? tab[kmax + 1].r : kInf;
        rmax = a < 0.0 ? (b + sq) / (-2.0 * a) : rh;
        rmax = rmax < rl ? rl : (rmax > rh ? rh : rmax);
      }

      // rejection sampling in s
      const double rc = 0.5 * (rmax + rmin), ra = 0.5 * (rmax - rmin);
      double r0 = rmin;
      double qacc = 0.0;
      bool have_q = false;
      int32_t ntr = 0;
      if (ra > 0.0) {
        const double glo = (J2 != 0.0) ? sqrt(2.0 * ra / fabs(dq_in(ms, kmin, rmin, J2))) : 0.0;
        const double ghi = sqrt(2.0 * ra / fabs(dq_in(ms, kmax, rmax, J2)));
        const double F = bound_factor * (glo > ghi ? glo : ghi);
        if (F > 0.0 && F < kInf) {
          bool accepted = false;
          for (int32_t j = 0; j < trial_cap; ++j) {
            const U4 w = philox(sid, step, kOrbit, static_cast<uint32_t>(j), seed);
            const double X = u01(w.y, w.x);
            const double X2 = u01(w.w, w.z);
            const double s0 = kPi * (X - 0.5);
            const double ss = sin(s0), cs = cos(s0);
            r0 = rc + ra * ss;
            ++ntr;
            const int64_t k0 = last_true(lv, n, RBelow{r0, kmin, kmax});
            const double q0 = 2.0 * E - 2.0 * phi_in(lv, ms, k0, r0) - J2 / (r0 * r0);
            if (!(q0 > 0.0)) continue;
            const double g0 = ra * cs / sqrt(q0);
            if (g0 > F) {
              c_viol += 1.0;
              fl |= CMC_ST_BOUND;
            }
            if (F * X2 < g0) {
              accepted = true;
              qacc = q0;  // Q at the accepted radius, reused for v_r
              have_q = true;
              break;
            }
          }
          if (!accepted) {
            c_cap = 1.0;
            fl |= CMC_ST_TRIAL_CAP;
          }
        } else {
          r0 = rc;
          fl |= CMC_ST_NUMERIC;
        }
      }
      c_tr = static_cast<double>(ntr);

      // new state: J conserved, E conserved in the old potential
      rn = r0 + 0.0;
      double qn = qacc;
      if (!have_q) {
        const int64_t kn = last_true(lv, n, RBelow{rn, kmin, kmax});
        qn = 2.0 * E - 2.0 * phi_in(lv, ms, kn, rn) - (J2 == 0.0 ? 0.0 : J2 / (rn * rn));
      }
      const U4 w = philox(sid, step, kSign, 0u, seed);
      const double vmag = sqrt(qn > 0.0 ? qn : 0.0);
      vrn = (w.x >> 31) ? -vmag : vmag;
      vtn = (J2 == 0.0) ? 0.0 : J / rn;
      if (!isfinite(rn) || !isfinite(vrn) || !isfinite(vtn)) fl |= CMC_ST_NONFINITE;
    }
    if (TO_STAGE) {
      StageRec rec;
      rec.r = rn;
      rec.vr = vrn;
      rec.vt = vtn;
      rec.m = load_mass(m, i);
      rec.id = sid;
      rec.pad = 0u;
      stage[i] = rec;
      keys[i] = __builtin_bit_cast(uint64_t, rn + 0.0);
    } else {
      r_new[i] = rn;
      vr[i] = vrn;
      vt[i] = vtn;
    }
  }

  // per-pass counters: block partials, summed in block order by k_orbit_sum
  if (__ballot(fl != 0)) {
    uint32_t wf = fl;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wf |= __shfl_xor(wf, o, 64);
    if ((threadIdx.x & 63) == 0 && wf) atomicOr(&sc->status, wf);
  }
  c_esc = block_sum<NT>(c_esc, shd);
  c_tr = block_sum<NT>(c_tr, shd);
  c_viol = block_sum<NT>(c_viol, shd);
  c_cap = block_sum<NT>(c_cap, shd);
  e_esc = block_sum<NT>(e_esc, shd);
  if (threadIdx.x == 0) {
    double *pp = part + 5 * static_cast<int64_t>(blockIdx.x);
    pp[0] = c_esc;
    pp[1] = c_tr;
    pp[2] = c_viol;
    pp[3] = c_cap;
    pp[4] = e_esc;
  }
}

constexpr int FT = 1024;

__global__ __launch_bounds__(FT) void k_orbit_sum(const double *__restrict__ part,
                                                  int64_t nblocks, cmc_scalars *__restrict__ sc) {
  __shared__ double sh[FT / 64];
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t b = threadIdx.x; b < nblocks; b += FT)
#pragma unroll
    for (int q = 0; q < 5; ++q) v[q] += part[5 * b + q];
#pragma unroll
  for (int q = 0; q < 5; ++q) v[q] = block_sum<FT>(v[q], sh);
  if (threadIdx.x == 0) {
    sc->n_esc = static_cast<int64_t>(v[0]);
    sc->trials = static_cast<int64_t>(v[1]);
    sc->violations = static_cast<int64_t>(v[2]);
    sc->capped = static_cast<int64_t>(v[3]);
    sc->e_esc = v[4];
  }
}

// The standalone orbit call reads the state's phi, mcum, ssuf: pack them into
// the table layout first.
__global__ __launch_bounds__(NT) void k_table_pack(const double *__restrict__ r,
                                                   const double *__restrict__ phi,
                                                   const double *__restrict__ mcum,
                                                   const double *__restrict__ ssuf,
                                                   const cmc_scalars *__restrict__ sc, Levels lv,
                                                   MS *__restrict__ ms) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
  if (k >= sc->n) return;
  put_table(lv, ms, k, r[k], phi[k], mcum[k], ssuf[k]);
}

template <typename MT>
hipError_t run(const cmc_state &s, const Workspace &w, const cmc_params &p, bool to_stage,
               hipStream_t st) {
  const MT *m = static_cast<const MT *>(s.m);
  const unsigned nb = static_cast<unsigned>(w.star_blocks);
  const int32_t cap = p.trial_cap > 0 ? p.trial_cap : 10000;
  const double bf = p.bound_factor > 0.0 ? p.bound_factor : 1.2;
  const Levels lv = levels_of(w);
  if (to_stage)
    k_orbit<MT, true><<<nb, NT, 0, st>>>(lv, w.ms, m, s.vr, s.vt, s.id, s.r_new, w.stage,
                                         w.keys[0], s.sc, w.red_part, p.seed, p.step, cap, bf);
  else
    k_orbit<MT, false><<<nb, NT, 0, st>>>(lv, w.ms, m, s.vr, s.vt, s.id, s.r_new, w.stage,
                                          w.keys[0], s.sc, w.red_part, p.seed, p.step, cap, bf);
  k_orbit_sum<<<1, FT, 0, st>>>(w.red_part, w.star_blocks, s.sc);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_table_pack(const cmc_state &s, const Workspace &w, hipStream_t st) {
  k_table_pack<<<static_cast<unsigned>(w.star_blocks), NT, 0, st>>>(s.r, s.phi, s.mcum, s.ssuf,
                                                                    s.sc, levels_of(w), w.ms);
  return hipGetLastError();
}

hipError_t launch_orbit(const cmc_state &s, const Workspace &w, const cmc_params &p,
                        bool to_stage, hipStream_t st) {
  return s.m_f32 ? run<float>(s, w, p, to_stage, st) : run<double>(s, w, p, to_stage, st);
}

}  // namespace cmc

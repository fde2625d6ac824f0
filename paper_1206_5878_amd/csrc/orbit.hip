// orbit.hip -- new orbits (arXiv:1206.5878, Sec. 2.1 step 5).  One thread per
// star: E = Phi_i + v^2/2 and J = r_i vt_i; the turning points are bracketed
// between table radii by bisection on the sign of Q_k = 2E - 2Phi_k - J^2/r_k^2
// (negative, positive, negative over k), solved in the bracket from
// r^2 Q = 2(E + S_k) r^2 + 2 M_k r - J^2; the new radius is drawn with density
// ~ 1/|v_r| by rejection in r = r_c + r_a sin s, where the density in s,
// g(s) = r_a cos s / sqrt(Q), is finite at both turning points.  The table
// (r, Phi, M, S) is read-only for the whole pass (old potential).
#include "cmc_internal.hpp"

namespace cmc {
namespace {

constexpr int NT = kBlock;

__device__ __forceinline__ double ld_coherent(const double *p) {
  const uint64_t u = __hip_atomic_load(reinterpret_cast<const uint64_t *>(p),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __builtin_bit_cast(double, u);
}

// Last table index k in [klo, khi] with r_k <= x.
__device__ __forceinline__ int64_t interval_of(const double *__restrict__ r, int64_t klo,
                                               int64_t khi, double x) {
  int64_t lo = klo, hi = khi + 1;
  while (hi - lo > 1) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (r[mid] <= x)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

__device__ __forceinline__ double phi_in(const double *__restrict__ phi,
                                         const double *__restrict__ mcum,
                                         const double *__restrict__ ssuf, int64_t k, double x) {
  if (k < 0) return phi[0];
  return -(mcum[k] / x + ssuf[k]);
}

__device__ __forceinline__ double dq_in(const double *__restrict__ mcum, int64_t k, double x,
                                        double J2) {
  const double grav = (k >= 0) ? -2.0 * mcum[k] / (x * x) : 0.0;
  return grav + 2.0 * J2 / (x * x * x);
}

template <typename MT, bool TO_STAGE>
__global__ __launch_bounds__(NT) void k_orbit(
    const double *__restrict__ r, const double *__restrict__ phi,
    const double *__restrict__ mcum, const double *__restrict__ ssuf,
    const MT *__restrict__ m, double *__restrict__ vr, double *__restrict__ vt,
    const uint32_t *__restrict__ id, double *__restrict__ r_new, StageRec *__restrict__ stage,
    uint64_t *__restrict__ keys, cmc_scalars *__restrict__ sc, double *__restrict__ part, uint32_t *__restrict__ ticket,
    uint64_t seed, uint32_t step, int32_t trial_cap, double bound_factor) {
  __shared__ double shd[NT / 64];
  __shared__ uint32_t is_last;
  const int64_t n = sc->n;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
  double c_esc = 0.0, c_tr = 0.0, c_viol = 0.0, c_cap = 0.0, e_esc = 0.0;
  uint32_t fl = 0;

  if (i < n) {
    const double vri = vr[i], vti = vt[i], ri = r[i];
    const double E = phi[i] + 0.5 * (vri * vri + vti * vti);
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
      // brackets
      int64_t lo = -1, hi = i;
      while (hi - lo > 1) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        const double rk = r[mid];
        if (2.0 * E - 2.0 * phi[mid] - J2 / (rk * rk) < 0.0)
          lo = mid;
        else
          hi = mid;
      }
      const int64_t kmin = lo;
      lo = i;
      hi = n;
      while (hi - lo > 1) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        const double rk = r[mid];
        if (2.0 * E - 2.0 * phi[mid] - J2 / (rk * rk) >= 0.0)
          lo = mid;
        else
          hi = mid;
      }
      const int64_t kmax = lo;

      // roots
      double rmin, rmax;
      if (J2 == 0.0) {
        rmin = 0.0;
      } else if (kmin < 0) {
        rmin = J / sqrt(2.0 * (E - phi[0]));
      } else {
        const double a = 2.0 * (E + ssuf[kmin]);
        const double b = 2.0 * mcum[kmin];
        const double disc = b * b + 4.0 * a * J2;
        const double den = b + sqrt(disc > 0.0 ? disc : 0.0);
        rmin = den > 0.0 ? 2.0 * J2 / den : r[kmin];
      }
      {
        const double rl = kmin >= 0 ? r[kmin] : 0.0, rh = r[kmin + 1];
        rmin = rmin < rl ? rl : (rmin > rh ? rh : rmin);
      }
      {
        const double a = 2.0 * (E + ssuf[kmax]);
        const double b = 2.0 * mcum[kmax];
        const double disc = b * b + 4.0 * a * J2;
        const double sq = sqrt(disc > 0.0 ? disc : 0.0);
        const double rh = (kmax + 1 < n) ? r[kmax + 1] : kInf;
        rmax = a < 0.0 ? (b + sq) / (-2.0 * a) : rh;
        const double rl = r[kmax];
        rmax = rmax < rl ? rl : (rmax > rh ? rh : rmax);
      }

      // rejection sampling in s
      const double rc = 0.5 * (rmax + rmin), ra = 0.5 * (rmax - rmin);
      double r0 = rmin;
      int32_t ntr = 0;
      if (ra > 0.0) {
        const double glo = (J2 != 0.0) ? sqrt(2.0 * ra / fabs(dq_in(mcum, kmin, rmin, J2))) : 0.0;
        const double ghi = sqrt(2.0 * ra / fabs(dq_in(mcum, kmax, rmax, J2)));
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
            const int64_t k0 = interval_of(r, kmin, kmax, r0);
            const double q0 = 2.0 * E - 2.0 * phi_in(phi, mcum, ssuf, k0, r0) - J2 / (r0 * r0);
            if (!(q0 > 0.0)) continue;
            const double g0 = ra * cs / sqrt(q0);
            if (g0 > F) {
              c_viol += 1.0;
              fl |= CMC_ST_BOUND;
            }
            if (F * X2 < g0) {
              accepted = true;
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
      const int64_t kn = interval_of(r, kmin, kmax, rn);
      const double qn = 2.0 * E - 2.0 * phi_in(phi, mcum, ssuf, kn, rn) -
                        (J2 == 0.0 ? 0.0 : J2 / (rn * rn));
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

  // per-pass counters: block partials, summed in block order by the last block
  const uint64_t any = __ballot(fl != 0);
  if (any) {
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
    __threadfence();
    const uint32_t tk = atomicAdd(ticket, 1u);
    is_last = (tk == gridDim.x - 1) ? 1u : 0u;
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t b = threadIdx.x; b < gridDim.x; b += NT)
    for (int q = 0; q < 5; ++q) v[q] += ld_coherent(part + 5 * b + q);
  for (int q = 0; q < 5; ++q) v[q] = block_sum<NT>(v[q], shd);
  if (threadIdx.x == 0) {
    ticket[0] = 0u;
    sc->n_esc = static_cast<int64_t>(v[0]);
    sc->trials = static_cast<int64_t>(v[1]);
    sc->violations = static_cast<int64_t>(v[2]);
    sc->capped = static_cast<int64_t>(v[3]);
    sc->e_esc = v[4];
  }
}

template <typename MT>
hipError_t run(const cmc_state &s, const Workspace &w, const cmc_params &p, bool to_stage,
               hipStream_t st) {
  const MT *m = static_cast<const MT *>(s.m);
  const unsigned nb = static_cast<unsigned>(w.star_blocks);
  const int32_t cap = p.trial_cap > 0 ? p.trial_cap : 10000;
  const double bf = p.bound_factor > 0.0 ? p.bound_factor : 1.2;
  if (to_stage)
    k_orbit<MT, true><<<nb, NT, 0, st>>>(s.r, s.phi, s.mcum, s.ssuf, m, s.vr, s.vt, s.id,
                                         s.r_new, w.stage, w.keys[0], s.sc, w.red_part,
                                         w.red_ticket,
                                         p.seed, p.step, cap, bf);
  else
    k_orbit<MT, false><<<nb, NT, 0, st>>>(s.r, s.phi, s.mcum, s.ssuf, m, s.vr, s.vt, s.id,
                                          s.r_new, w.stage, w.keys[0], s.sc, w.red_part,
                                          w.red_ticket,
                                          p.seed, p.step, cap, bf);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_orbit(const cmc_state &s, const Workspace &w, const cmc_params &p,
                        bool to_stage, hipStream_t st) {
  return s.m_f32 ? run<float>(s, w, p, to_stage, st) : run<double>(s, w, p, to_stage, st);
}

}  // namespace cmc

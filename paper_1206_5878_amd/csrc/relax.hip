// relax.hip -- shared timestep and two-body relaxation (arXiv:1206.5878,
// Sec. 2.1 steps 2-3, Sec. 3.2 bins).  Neighbour pairs (2p, 2p+1); local
// number density from the pair's 20-star radial bin; representative-encounter
// time t_p = (pi/32) w^3 / (lnL n_b (m1+m2)^2); deflection
// beta = min(pi, (pi/2) sqrt(dt/t_p)).  dt solves mean_p sin^2(beta_p/2) =
// target by safeguarded Newton on x = ln dt: per iteration one grid-wide
// evaluation and a one-block update.  One thread per pair otherwise.  A
// pair's random block comes from Philox or from its first star's LFSR113
// stream (Sec. 3.6), which only the kick advances.  The
// mixed form computes the pair terms and the kick in FP32 and keeps the
// centre-of-mass velocity, the sums and the Newton solve in FP64.
#include <type_traits>

#include "cmc_internal.hpp"

namespace cmc {
namespace {

constexpr int NT = kBlock;

struct PairGeo {
  double v1x, v1y, v2x, v2y, v2z, wx, wy, wz, wm, tp, u2, ma, mb;
};

// The pair's random block: Philox at counter (id of its first star, step,
// kRelax, 0), or the next block of the first star's LFSR113 stream (consume:
// advance the stream; the timestep's pass only reads it).
template <bool LF>
__device__ __forceinline__ U4 pair_block(const ClusterArgs &A, int64_t a, uint32_t step,
                                         bool consume) {
  if (!LF) return philox(A.s.id[a], step, kRelax, 0u, A.seed);
  Lfsr g = load_lfsr(A.s.rng, a);
  const U4 w = lfsr_block(g);
  if (consume) store_lfsr(A.s.rng, a, g);
  return w;
}

template <typename MT, bool MIXED>
__device__ __forceinline__ PairGeo pair_geometry(int64_t p, int64_t n,
                                                 const double *__restrict__ r,
                                                 const MT *__restrict__ m,
                                                 const double *__restrict__ vr,
                                                 const double *__restrict__ vt,
                                                 const U4 &w, double lnL) {
  PairGeo g;
  int64_t nbins = n / 20;
  if (nbins < 1) nbins = 1;
  const int64_t a = 2 * p, b = a + 1;
  int64_t bin = a / 20;
  if (bin > nbins - 1) bin = nbins - 1;
  const int64_t lo = 20 * bin;
  const int64_t hi = (bin == nbins - 1) ? n - 1 : 20 * bin + 19;
  const double rl = r[lo], rh = r[hi];
  const double vol = (4.0 * kPi / 3.0) * (rh - rl) * (rh * rh + rh * rl + rl * rl);
  const double nb = vol > 0.0 ? static_cast<double>(hi - lo) / vol : kInf;

  g.v1x = vr[a];
  g.v1y = vt[a];
  g.v2x = vr[b];
  g.ma = load_mass(m, a);
  g.mb = load_mass(m, b);
  const double ms = g.ma + g.mb;
  if (MIXED) {
    // pair terms in FP32 (psi from the 23-bit uniform)
    g.u2 = static_cast<double>(u01f(w.w));
    float sp, cp;
    sincosf(2.0f * static_cast<float>(kPi) * u01f(w.y), &sp, &cp);
    const float vtb = static_cast<float>(vt[b]);
    const float v2y = vtb * cp, v2z = vtb * sp;
    const float wx = static_cast<float>(g.v1x - g.v2x);
    const float wy = static_cast<float>(g.v1y) - v2y;
    const float wz = -v2z;
    const float wm = sqrtf(wx * wx + wy * wy + wz * wz);
    g.v2y = v2y;
    g.v2z = v2z;
    g.wx = wx;
    g.wy = wy;
    g.wz = wz;
    g.wm = wm;
    if (ms == 0.0 || lnL == 0.0)
      g.tp = kInf;
    else if (isinf(nb))
      g.tp = 0.0;
    else {
      const float msf = static_cast<float>(ms);
      g.tp = static_cast<double>((static_cast<float>(kPi) / 32.0f) * (wm * wm * wm) /
                                 (static_cast<float>(lnL) * static_cast<float>(nb) * (msf * msf)));
    }
    return g;
  }
  const double u1 = u01(w.y, w.x);
  g.u2 = u01(w.w, w.z);
  const double psi = 2.0 * kPi * u1;
  double sp, cp;
  sincos(psi, &sp, &cp);
  g.v2y = vt[b] * cp;
  g.v2z = vt[b] * sp;
  g.wx = g.v1x - g.v2x;
  g.wy = g.v1y - g.v2y;
  g.wz = 0.0 - g.v2z;
  g.wm = sqrt(g.wx * g.wx + g.wy * g.wy + g.wz * g.wz);
  if (ms == 0.0 || lnL == 0.0)
    g.tp = kInf;
  else if (isinf(nb))
    g.tp = 0.0;
  else
    g.tp = (kPi / 32.0) * (g.wm * g.wm * g.wm) / (lnL * nb * (ms * ms));
  return g;
}

__device__ __forceinline__ double coulomb_log(double gamma, int64_t n) {
  const double l = log(gamma * static_cast<double>(n));
  return l > 0.0 ? l : 0.0;
}

__device__ __forceinline__ double beta_of(double tp, double dt) {
  if (!(dt > 0.0) || isinf(tp)) return 0.0;
  if (tp == 0.0) return kPi;
  const double b = 0.5 * kPi * sqrt(dt / tp);
  return b < kPi ? b : kPi;
}

// ---------------------------------------------------------------- timestep
// dt_state slots
enum { kX = 0, kLo, kHi, kDone, kIt, kCnt, kZero, kInfN, kLogSum };

template <class Ctx, typename MT, bool MIXED, bool LF>
__global__ __launch_bounds__(NT) void k_pair_tp(Ctx ctx, uint32_t step_arg) {
  __shared__ double sh[4 * (NT / 64)];
  const ClusterArgs &A = ctx.args();
  const uint32_t step = step_of(A, step_arg);
  const double *__restrict__ r = A.s.r;
  const MT *__restrict__ m = static_cast<const MT *>(A.s.m);
  const double *__restrict__ vr = A.s.vr;
  const double *__restrict__ vt = A.s.vt;
  double *__restrict__ tp_out = A.w.pair_tp;
  double *__restrict__ part = A.w.pair_part;
  const double gamma = A.gamma;
  const int64_t n = A.s.sc->n;
  const int64_t np = n / 2;
  // the sum of ln t_p only seeds a cold start (no previous dt)
  const bool cold = !(A.s.sc->dt > 0.0);
  const int64_t blk = ctx.block();
  const int64_t p = blk * NT + threadIdx.x;
  double v[4] = {0.0, 0.0, 0.0, 0.0};  // counted, t_p = 0, t_p = inf, sum ln t_p
  if (p < np) {
    const U4 w = pair_block<LF>(A, 2 * p, step, false);
    const PairGeo g = pair_geometry<MT, MIXED>(p, n, r, m, vr, vt, w, coulomb_log(gamma, n));
    if (g.wm > 0.0) {
      // what the Newton evaluations need of t_p: beta = (pi/2) sqrt(dt) u
      // with u = t_p^-1/2 (+inf for t_p = 0, 0 for t_p = inf); FP32 in the
      // mixed form, whose t_p is an FP32 value
      if (MIXED) {
        const float tf = static_cast<float>(g.tp);
        reinterpret_cast<float *>(tp_out)[p] =
            tf == 0.0f ? kInfF : (isinf(tf) ? 0.0f : 1.0f / sqrtf(tf));
      } else {
        tp_out[p] = g.tp == 0.0 ? kInf : (isinf(g.tp) ? 0.0 : 1.0 / sqrt(g.tp));
      }
      v[0] = 1.0;
      if (g.tp == 0.0)
        v[1] = 1.0;
      else if (isinf(g.tp))
        v[2] = 1.0;
      else if (cold)
        v[3] = log(g.tp);
    } else if (MIXED) {
      reinterpret_cast<float *>(tp_out)[p] = -1.0f;  // no relative motion: not counted
    } else {
      tp_out[p] = -1.0;
    }
  }
  // the four block sums through one LDS exchange (wave order, then waves)
#pragma unroll
  for (int q = 0; q < 4; ++q) v[q] = wave_sum(v[q]);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < 4; ++q) sh[4 * w + q] = v[q];
  __syncthreads();
  if (threadIdx.x < 4) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) t += sh[4 * i + threadIdx.x];
    part[4 * blk + threadIdx.x] = t;
  }
}

constexpr int IT = 1024;

// Reduce the pair counts, detect the degenerate cases, pick the start point.
// One block per cluster.
template <class Ctx>
__global__ __launch_bounds__(IT) void k_dt_init(Ctx ctx, double target) {
  __shared__ double sh[IT / 64];
  const ClusterArgs &A = ctx.args();
  const double *__restrict__ part = A.w.pair_part;
  const int64_t nblocks = A.w.pair_blocks;
  double *__restrict__ st = A.w.dt_state;
  cmc_scalars *__restrict__ sc = A.s.sc;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int64_t b = threadIdx.x; b < nblocks; b += IT)
    for (int q = 0; q < 4; ++q) v[q] += part[4 * b + q];
  for (int q = 0; q < 4; ++q) v[q] = block_sum<IT>(v[q], sh);
  if (threadIdx.x == 0) {
    const double cnt = v[0], nz = v[1], ni = v[2], ls = v[3];
    st[kCnt] = cnt;
    st[kZero] = nz;
    st[kInfN] = ni;
    st[kIt] = 0.0;
    st[kLo] = -kInf;
    st[kHi] = kInf;
    if (cnt == 0.0 || nz / cnt >= target || (cnt - ni) / cnt <= target) {
      st[kDone] = 1.0;
      st[kX] = -kInf;
      sc->dt = 0.0;
      sc->dt_iters = 0u;
      atomicOr(&sc->status, CMC_ST_DT_DEGEN);
      return;
    }
    double x;
    if (sc->dt > 0.0) {
      x = log(sc->dt);
    } else {
      // small angles: mean sin^2(beta/2) ~ (pi^2/16) dt <1/t_p>; use the
      // geometric mean of the finite t_p for <1/t_p>^-1
      const double nf = cnt - nz - ni;
      x = log(16.0 * target / (kPi * kPi)) + (nf > 0.0 ? ls / nf : 0.0);
    }
    st[kX] = x;
    st[kDone] = 0.0;
  }
}

// sin^2(beta/2) and its derivative d/dx = (1/4) beta sin(beta) (beta < pi) for
// one pair, beta = min(pi, c u) with c = (pi/2) sqrt(dt) > 0 (u < 0: a pair
// that is not counted).
template <bool MIXED>
__device__ __forceinline__ void dt_terms(double u, double c, double &h, double &d) {
  if (!(u >= 0.0)) return;
  const double bu = isinf(u) ? kPi : c * u;
  const double b = bu < kPi ? bu : kPi;
  if (MIXED) {  // per-pair terms in FP32, sums in FP64
    const float bf = static_cast<float>(b);
    float sf, cf;
    sincosf(0.5f * bf, &sf, &cf);
    h += static_cast<double>(sf * sf);
    if (b < kPi) d += static_cast<double>(0.5f * bf * sf * cf);
  } else {
    double sn, cs;
    sincos(0.5 * b, &sn, &cs);
    h += sn * sn;
    if (b < kPi) d += 0.5 * b * sn * cs;
  }
}

// One Newton evaluation: block partials of sum sin^2(beta/2) and of its
// derivative at dt = exp(x), from each pair's t_p^-1/2.  Each thread keeps
// four loads in flight and adds its pairs in grid-stride order.
template <class Ctx, bool MIXED>
__global__ __launch_bounds__(NT) void k_dt_eval(Ctx ctx) {
  __shared__ double sh[NT / 64];
  const ClusterArgs &A = ctx.args();
  const double *__restrict__ st = A.w.dt_state;
  double *__restrict__ part = A.w.red_part;
  if (st[kDone] != 0.0) return;
  const int64_t np = A.s.sc->n / 2;
  const double c = 0.5 * kPi * sqrt(exp(st[kX]));
  const int64_t blk = ctx.block();
  const int64_t stride = ctx.nblocks() * NT;
  double h = 0.0, d = 0.0;
  for (int64_t p0 = blk * NT + threadIdx.x; p0 < np; p0 += 4 * stride) {
    double t[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t p = p0 + q * stride;
      t[q] = -1.0;
      if (p < np)
        t[q] = MIXED ? static_cast<double>(reinterpret_cast<const float *>(A.w.pair_tp)[p])
                     : A.w.pair_tp[p];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) dt_terms<MIXED>(t[q], c, h, d);
  }
  h = block_sum<NT>(h, sh);
  d = block_sum<NT>(d, sh);
  if (threadIdx.x == 0) {
    part[2 * blk + 0] = h;
    part[2 * blk + 1] = d;
  }
}

// Sum the partials in block order and take one safeguarded Newton step on
// G(x) = ln F(x) - ln target (dG/dx = F'/F), keeping a bracket [lo, hi] of the
// root; converged when the step falls below 1e-14 relative.
// One block per cluster; the partials are those of the cluster's k_dt_eval
// blocks.
template <class Ctx>
__global__ __launch_bounds__(NT) void k_dt_update(Ctx ctx, double target, double xtol,
                                                  int32_t last_iter) {
  __shared__ double sh[NT / 64];
  const ClusterArgs &A = ctx.args();
  const double *__restrict__ part = A.w.red_part;
  const int64_t nblocks = A.w.pair_blocks < kRedBlocks ? A.w.pair_blocks : kRedBlocks;
  double *__restrict__ st = A.w.dt_state;
  cmc_scalars *__restrict__ sc = A.s.sc;
  if (st[kDone] != 0.0) return;
  double H = 0.0, D = 0.0;
  for (int64_t b = threadIdx.x; b < nblocks; b += NT) {
    H += part[2 * b];
    D += part[2 * b + 1];
  }
  H = block_sum<NT>(H, sh);
  D = block_sum<NT>(D, sh);
  if (threadIdx.x != 0) return;
  const double x = st[kX];
  const double cnt = st[kCnt];
  const double F = H / cnt, Fp = D / cnt;
  double lo = st[kLo], hi = st[kHi];
  if (F < target)
    lo = x;
  else
    hi = x;
  bool conv = (F == target);
  double xn = x;
  if (!conv) {
    xn = (F > 0.0 && Fp > 0.0) ? x - log(F / target) * F / Fp : __builtin_nan("");
    const double tol = xtol * fmax(1.0, fabs(x));
    // a Newton step this small is done, even when it rounds back onto x (which
    // may coincide with the bracket end just moved there)
    if (fabs(xn - x) <= tol) {
      conv = true;
    } else {
      const bool closed = isfinite(lo) && isfinite(hi);
      if (!(xn > lo && xn < hi) || (!closed && fabs(xn - x) > 16.0)) {
        if (closed)
          xn = 0.5 * (lo + hi);
        else
          xn = (F < target) ? x + 8.0 : x - 8.0;
      }
      if (closed && hi - lo <= 1e-15 * fmax(1.0, fabs(x))) conv = true;
    }
  }
  const double it = st[kIt] + 1.0;
  st[kIt] = it;
  st[kLo] = lo;
  st[kHi] = hi;
  st[kX] = xn;
  st[kDone] = conv ? 1.0 : 0.0;
  sc->dt = exp(xn);
  sc->dt_iters = static_cast<uint32_t>(it);
  if (!conv && last_iter) atomicOr(&sc->status, CMC_ST_DT_NOCONV);
}

// ---------------------------------------------------------------- kicks
template <class Ctx, typename MT, bool MIXED, bool LF>
__global__ __launch_bounds__(NT) void k_relax(Ctx ctx, uint32_t step_arg) {
  const ClusterArgs &A = ctx.args();
  const uint32_t step = step_of(A, step_arg);
  const double *__restrict__ r = A.s.r;
  const MT *__restrict__ m = static_cast<const MT *>(A.s.m);
  double *__restrict__ vr = A.s.vr;
  double *__restrict__ vt = A.s.vt;
  const double gamma = A.gamma;
  const int64_t n = A.s.sc->n;
  const int64_t np = n / 2;
  const int64_t p = ctx.block() * NT + threadIdx.x;
  if (p >= np) return;
  const double dt = A.s.sc->dt;
  const U4 w = pair_block<LF>(A, 2 * p, step, true);  // every pair draws, kicked or not
  const PairGeo g = pair_geometry<MT, MIXED>(p, n, r, m, vr, vt, w, coulomb_log(gamma, n));
  const double beta = beta_of(g.tp, dt);
  if (!(g.wm > 0.0) || beta == 0.0) return;
  const int64_t a = 2 * p, b = a + 1;
  if (MIXED) {
    // the kick in FP32, the centre of mass and the new velocities in FP64
    const float wm = static_cast<float>(g.wm);
    const float wx = static_cast<float>(g.wx), wy = static_cast<float>(g.wy),
                wz = static_cast<float>(g.wz);
    const float e1x = wx / wm, e1y = wy / wm, e1z = wz / wm;
    const float ax = fabsf(wx), ay = fabsf(wy), az = fabsf(wz);
    float cx, cy, cz;
    if (ax <= ay && ax <= az) {
      cx = 0.0f;
      cy = e1z;
      cz = -e1y;
    } else if (ay <= az) {
      cx = -e1z;
      cy = 0.0f;
      cz = e1x;
    } else {
      cx = e1y;
      cy = -e1x;
      cz = 0.0f;
    }
    const float cn = sqrtf(cx * cx + cy * cy + cz * cz);
    const float e2x = cx / cn, e2y = cy / cn, e2z = cz / cn;
    const float e3x = e1y * e2z - e1z * e2y;
    const float e3y = e1z * e2x - e1x * e2z;
    const float e3z = e1x * e2y - e1y * e2x;
    float sb, cb, s2, c2;
    sincosf(static_cast<float>(beta), &sb, &cb);
    sincosf(2.0f * static_cast<float>(kPi) * static_cast<float>(g.u2), &s2, &c2);
    const float wnx = wm * (cb * e1x + sb * (c2 * e2x + s2 * e3x));
    const float wny = wm * (cb * e1y + sb * (c2 * e2y + s2 * e3y));
    const float wnz = wm * (cb * e1z + sb * (c2 * e2z + s2 * e3z));
    const double ims = 1.0 / (g.ma + g.mb);
    const double fa = g.ma * ims, fb = g.mb * ims;
    const double cmx = fa * g.v1x + fb * g.v2x;
    const double cmy = fa * g.v1y + fb * g.v2y;
    const double cmz = fb * g.v2z;
    const double n1x = cmx + fb * wnx, n1y = cmy + fb * wny, n1z = cmz + fb * wnz;
    const double n2x = cmx - fa * wnx, n2y = cmy - fa * wny, n2z = cmz - fa * wnz;
    vr[a] = n1x;
    vt[a] = sqrt(n1y * n1y + n1z * n1z);
    vr[b] = n2x;
    vt[b] = sqrt(n2y * n2y + n2z * n2z);
    return;
  }

  const double iwm = 1.0 / g.wm;
  const double e1x = g.wx * iwm, e1y = g.wy * iwm, e1z = g.wz * iwm;
  const double ax = fabs(g.wx), ay = fabs(g.wy), az = fabs(g.wz);
  double cx, cy, cz;  // e1 x (axis of the smallest |w| component)
  if (ax <= ay && ax <= az) {
    cx = 0.0;
    cy = e1z;
    cz = -e1y;
  } else if (ay <= az) {
    cx = -e1z;
    cy = 0.0;
    cz = e1x;
  } else {
    cx = e1y;
    cy = -e1x;
    cz = 0.0;
  }
  const double icn = 1.0 / sqrt(cx * cx + cy * cy + cz * cz);
  const double e2x = cx * icn, e2y = cy * icn, e2z = cz * icn;
  const double e3x = e1y * e2z - e1z * e2y;
  const double e3y = e1z * e2x - e1x * e2z;
  const double e3z = e1x * e2y - e1y * e2x;
  const double psi2 = 2.0 * kPi * g.u2;
  double sb, cb, s2, c2;
  sincos(beta, &sb, &cb);
  sincos(psi2, &s2, &c2);
  const double wnx = g.wm * (cb * e1x + sb * (c2 * e2x + s2 * e3x));
  const double wny = g.wm * (cb * e1y + sb * (c2 * e2y + s2 * e3y));
  const double wnz = g.wm * (cb * e1z + sb * (c2 * e2z + s2 * e3z));
  const double ims = 1.0 / (g.ma + g.mb);
  const double fa = g.ma * ims, fb = g.mb * ims;
  const double cmx = fa * g.v1x + fb * g.v2x;
  const double cmy = fa * g.v1y + fb * g.v2y;
  const double cmz = fa * 0.0 + fb * g.v2z;
  const double n1x = cmx + fb * wnx, n1y = cmy + fb * wny, n1z = cmz + fb * wnz;
  const double n2x = cmx - fa * wnx, n2y = cmy - fa * wny, n2z = cmz - fa * wnz;
  // |v_t| from its two components (O(1) speeds: no overflow to guard against)
  vr[a] = n1x;
  vt[a] = sqrt(n1y * n1y + n1z * n1z);
  vr[b] = n2x;
  vt[b] = sqrt(n2y * n2y + n2z * n2z);
}

template <class L, typename MT, bool MIXED>
hipError_t run_timestep(const L &l, const cmc_params &p, hipStream_t st) {
  // Newton stops once its step in ln dt is below what the terms resolve:
  // FP64 terms to ~1e-16, FP32 terms (mixed) to ~1e-7 each
  const double kXTol = MIXED ? 1e-7 : 1e-14;
  if (p.rng == CMC_RNG_LFSR113)
    k_pair_tp<decltype(l.ctx(kShPair)), MT, MIXED, true><<<l.grid(kShPair), NT, 0, st>>>(
        l.ctx(kShPair), p.step);
  else
    k_pair_tp<decltype(l.ctx(kShPair)), MT, MIXED, false><<<l.grid(kShPair), NT, 0, st>>>(
        l.ctx(kShPair), p.step);
  k_dt_init<<<l.grid(kShOne), IT, 0, st>>>(l.ctx(kShOne), p.target);
  const int iters = p.dt_iters > 0 ? p.dt_iters : 10;
  for (int i = 0; i < iters; ++i) {
    k_dt_eval<decltype(l.ctx(kShDtEval)), MIXED><<<l.grid(kShDtEval), NT, 0, st>>>(
        l.ctx(kShDtEval));
    k_dt_update<<<l.grid(kShOne), NT, 0, st>>>(l.ctx(kShOne), p.target, kXTol,
                                               i == iters - 1 ? 1 : 0);
  }
  return hipGetLastError();
}

template <class L, typename MT, bool MIXED>
hipError_t run_relax(const L &l, const cmc_params &p, hipStream_t st) {
  if (p.rng == CMC_RNG_LFSR113)
    k_relax<decltype(l.ctx(kShPair)), MT, MIXED, true><<<l.grid(kShPair), NT, 0, st>>>(
        l.ctx(kShPair), p.step);
  else
    k_relax<decltype(l.ctx(kShPair)), MT, MIXED, false><<<l.grid(kShPair), NT, 0, st>>>(
        l.ctx(kShPair), p.step);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_timestep(const Target &t, bool m_f32, const cmc_params &p, hipStream_t st) {
  return dispatch(t, [&](const auto &l) {
    using L = std::decay_t<decltype(l)>;
    const bool mx = p.precision == CMC_MIXED;
    if (m_f32)
      return mx ? run_timestep<L, float, true>(l, p, st) : run_timestep<L, float, false>(l, p, st);
    return mx ? run_timestep<L, double, true>(l, p, st) : run_timestep<L, double, false>(l, p, st);
  });
}

hipError_t launch_relax(const Target &t, bool m_f32, const cmc_params &p, hipStream_t st) {
  return dispatch(t, [&](const auto &l) {
    using L = std::decay_t<decltype(l)>;
    const bool mx = p.precision == CMC_MIXED;
    if (m_f32)
      return mx ? run_relax<L, float, true>(l, p, st) : run_relax<L, float, false>(l, p, st);
    return mx ? run_relax<L, double, true>(l, p, st) : run_relax<L, double, false>(l, p, st);
  });
}

}  // namespace cmc

// orbit.hip -- new orbits (arXiv:1206.5878, Sec. 2.1 step 5).  Per star:
// E = Phi_i + v^2/2 and J = r_i vt_i; the turning points are bracketed
// between table radii by the sign of Q_k = 2E - 2Phi_k - J^2/r_k^2 (negative,
// positive, negative over k), solved in the bracket from
// r^2 Q = 2(E + S_k) r^2 + 2 M_k r - J^2; the new radius is drawn with density
// ~ 1/|v_r| by rejection in r = r_c + r_a sin s, where the density in s,
// g(s) = r_a cos s / sqrt(Q), is finite at both turning points.  The table
// is read-only for the whole pass (old potential).
//
// The mixed form draws the trial angle and takes the accept test in FP32;
// brackets, roots, the table and Q stay in FP64.
//
// For the energy correction of Sec. 2.1 item 6 (energy.hip) a step can also
// record, per star in this pass's order, (r_old, Phi_old(r_old)) and the old
// potential at the new radius, Phi_old(r_new).  Draws come from Philox or,
// with the LFSR113 generator of Sec. 3.6, from the star's own stream, whose
// state then leaves with the staged star.
//
// Two kernels.  k_orbit_bracket: brackets, roots and the rejection bound F
// of every star, written as a 48-byte orbit record (escapers and degenerate
// orbits are finished there); its blocks stay resident and loop over tiles
// of stars.  k_orbit_trials: each wavefront owns a chunk of stars and every
// lane draws trials for one star at a time, taking the chunk's next star as
// soon as its own is accepted, so the loop does not wait for the unluckiest
// lane of the wavefront.
//
// Searches.  The lower and the upper bracket are each "the last index k
// where a predicate monotone in k holds".  They descend the sampled levels of
// the table (level L = every 8^L-th (r, Phi)): per level, the 8 children of
// the current sample are one aligned cache line, and the count of children
// that satisfy the predicate is the next sample.  The top levels (a few
// thousand entries) sit in LDS and each lane descends them alone; below
// them, lanes work in groups of 8 so that every node is one coalesced load.
// Brackets are unique, so this finds the index a bisection over the whole
// table finds.  The interval of a trial radius comes from the radial bucket
// index (rindex.hip); a trial that the potential-bound table proves rejected
// skips that lookup (see surely_rejected).
#include <algorithm>
#include <type_traits>

#include "cmc_internal.hpp"

namespace cmc {
namespace {

constexpr int NT = kBlock;
constexpr int BT = 512;         // threads per block of the bracket kernel
constexpr int kChunk = 128;     // stars per wavefront in the trial kernel
// group searches whose loads are in flight together: 4 keeps the bracket
// kernel at 86 VGPRs without spills (8 needs 118); its occupancy is set by
// the LDS-resident top levels either way, and 4 measured ~1 % faster
constexpr int kGroupBatch = 4;
static_assert(16 % kGroupBatch == 0, "batches split the 16 searches of a group");

// Sign of Q_k = 2E - 2Phi_k - J^2/r_k^2 without the division:
// (2E - 2Phi_k) r_k^2 against J^2.  A star at r_k = 0 takes the limit r -> 0:
// Q = -inf when J != 0 (the J^2/r^2 term wins, even against Phi_k = -inf),
// else 2E - 2Phi_k.
__device__ __forceinline__ bool q_neg(double twoE, double J2, const RPhi &e) {
  if (e.r == 0.0) return J2 > 0.0 || twoE - 2.0 * e.phi < 0.0;
  return (twoE - 2.0 * e.phi) * (e.r * e.r) < J2;
}
__device__ __forceinline__ bool q_nonneg(double twoE, double J2, const RPhi &e) {
  if (e.r == 0.0) return J2 == 0.0 && twoE - 2.0 * e.phi >= 0.0;
  return (twoE - 2.0 * e.phi) * (e.r * e.r) >= J2;
}
// Q_k < 0 and k < below.
struct QNeg {
  double twoE, J2;
  int64_t below;
  __device__ bool operator()(int64_t k, const RPhi &e) const {
    return k < below && q_neg(twoE, J2, e);
  }
};
// Q_k >= 0 or k <= upto.
struct QNonNeg {
  double twoE, J2;
  int64_t upto;
  __device__ bool operator()(int64_t k, const RPhi &e) const {
    return k <= upto || q_nonneg(twoE, J2, e);
  }
};

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

// Interval of x for the potential: the last k with r_k <= x, kept inside the
// orbit's brackets [kmin, kmax].
__device__ __forceinline__ int64_t interval_in(const RIndex &ix, const RIndexCtl &c, double x,
                                               int64_t kmin, int64_t kmax) {
  const int64_t k = rindex_last_le(ix, c, x);
  return k < kmin ? kmin : (k > kmax ? kmax : k);
}

// ---------------------------------------------------------------- potential bounds
// Phi rises outward, so for edge radii x_b <= x < x_(b+1) the potential at a
// trial radius lies in [Phi(x_b), Phi(x_(b+1))].  The edges are equal steps of
// the IEEE bit pattern from r_0 (about equal steps in ln r), kPhiBins of them
// over the table's range; below r_0 the potential is Phi_0, beyond the last
// edge it lies in [Phi(last edge), 0].
struct PhiBounds {
  const double *tab;  // [kPhiBins + 1]
  uint64_t lo;        // bits of the first edge (r_0)
  uint32_t shift;
  double phi0;        // Phi_0
};

// Whether the trial at x is certainly rejected.  The bounds on Phi bound
// Q = 2E - 2 Phi - J^2/x^2 and the acceptance ratio g = r_a cos s / sqrt(Q);
// a rejection is called only when it holds with a margin far above the
// rounding of the exact test (relative 1e-12 on Q, 1e-12 on g in FP64, 1e-5
// on the FP32 g of the mixed form), so the exact test would reject as well,
// and the trial is counted the same way (no bound violation: g < F X2 < F).
template <bool MIXED>
__device__ __forceinline__ bool surely_rejected(const PhiBounds &pb, double x, double E,
                                                double J2, double ra, double cs, double F,
                                                double X2) {
  const uint64_t kx = rbits(x);
  double plo, phi;
  if (kx < pb.lo) {
    plo = phi = pb.phi0;
  } else {
    const uint64_t b = (kx - pb.lo) >> pb.shift;
    if (b >= static_cast<uint64_t>(kPhiBins)) {
      plo = pb.tab[kPhiBins];
      phi = 0.0;
    } else {
      plo = pb.tab[b];
      phi = pb.tab[b + 1];
    }
  }
  const double c2 = J2 / (x * x);
  const double mu = 1e-12 * (2.0 * fabs(E) + 2.0 * fabs(plo) + 2.0 * fabs(phi) + c2);
  const double qmax = 2.0 * E - 2.0 * plo - c2 + mu;
  if (qmax <= 0.0) return true;
  const double qmin = 2.0 * E - 2.0 * phi - c2 - mu;
  if (!(qmin > 0.0)) return false;
  const double gmax = ra * cs / sqrt(qmin);
  if (MIXED) {
    const float pf = static_cast<float>(F) * static_cast<float>(X2);
    return static_cast<double>(pf) >= gmax * (1.0 + 1e-5);
  }
  return F * X2 >= gmax * (1.0 + 1e-12);
}

// ---------------------------------------------------------------- group search
// The same search, cooperative: lanes form groups of 8 (group g = lanes
// 8g..8g+7), and each group runs the searches of its 8 lanes together.  Per
// level, lane q of the group loads child q of each of the 8 current samples,
// so every node is one coalesced 128-byte load instead of 7 loads per lane,
// and a ballot counts the children that satisfy the predicate.  Predicate
// parameters travel through LDS.  Every lane of the wavefront must call it.
struct GParams {
  double a, b;  // QNeg/QNonNeg: 2E, J^2
  int32_t c;    // QNeg: below; QNonNeg: upto
  int32_t s0;   // sample reached at level ltop (-1: no index holds)
};
struct GQNeg {
  __device__ static bool eval(const GParams &p, int64_t k, const RPhi &e) {
    return k < p.c && q_neg(p.a, p.b, e);
  }
};
struct GQNonNeg {
  __device__ static bool eval(const GParams &p, int64_t k, const RPhi &e) {
    return k <= p.c || q_nonneg(p.a, p.b, e);
  }
};

// Descent of the levels below ltop for two searches per lane (predicates PA
// and PB, e.g. the lower and the upper bracket).  Each lane brings the
// samples its own searches reached at level ltop (see top_descend; -1: no
// index holds).  All 16 searches of a group have their loads in flight
// together, so a level costs one memory round trip.
template <class PA, class PB>
__device__ __forceinline__ void group_descend2(const Levels &lv, int ltop, int64_t n,
                                               const GParams &ma, const GParams &mb,
                                               GParams *prm_a, GParams *prm_b, int64_t &ka,
                                               int64_t &kb) {
  const int lane = threadIdx.x & 63, g = lane >> 3, q = lane & 7;
  prm_a[lane] = ma;
  prm_b[lane] = mb;
  __builtin_amdgcn_wave_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  int32_t s[16];
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    s[t] = prm_a[(g << 3) + t].s0;
    s[8 + t] = prm_b[(g << 3) + t].s0;
  }
#pragma unroll
  for (int L = kMaxLevels - 1; L >= 0; --L) {
    if (L < ltop) {
      // re-read the parameters from LDS at every level rather than keep
      // 16 sets of them live in registers
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      const int64_t stride = int64_t(1) << (3 * L);
      const int64_t cnt = (n + stride - 1) / stride;
      const RPhi *lev = lv.lev[L];
#pragma unroll
      for (int h = 0; h < 16; h += kGroupBatch) {
        RPhi e[kGroupBatch];
#pragma unroll
        for (int v = 0; v < kGroupBatch; ++v) {
          const int u = h + v;
          const int64_t child = static_cast<int64_t>(s[u]) * 8 + q;
          e[v] = (s[u] >= 0 && child < cnt) ? lev[child] : RPhi{0.0, 0.0};
        }
#pragma unroll
        for (int v = 0; v < kGroupBatch; ++v) {
          const int u = h + v;
          const GParams p = (u < 8) ? prm_a[(g << 3) + u] : prm_b[(g << 3) + u - 8];
          const int64_t child = static_cast<int64_t>(s[u]) * 8 + q;
          const bool in = s[u] >= 0 && child < cnt;
          const bool ok = in && ((u < 8) ? PA::eval(p, child * stride, e[v])
                                         : PB::eval(p, child * stride, e[v]));
          const uint64_t m = __ballot(ok);
          const int c = __popcll((m >> (g << 3)) & 0xFFull);
          if (s[u] >= 0) s[u] = s[u] * 8 + c - 1;
        }
      }
    }
  }
  __builtin_amdgcn_wave_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  int32_t ra = s[0], rb = s[8];
#pragma unroll
  for (int t = 1; t < 8; ++t) {
    if (q == t) {
      ra = s[t];
      rb = s[8 + t];
    }
  }
  ka = ra;
  kb = rb;
}

// ---------------------------------------------------------------- LDS top
// The levels [ltop, nlev) -- a few thousand entries, see orbit_top() -- are
// copied into LDS by every block of the bracket kernel; each lane descends
// them on its own.
constexpr int kTopBytes = 48 * 1024;

template <class Pred>
__device__ __forceinline__ int32_t top_descend(const RPhi *top, const OrbitTop &tl, int nlev,
                                               int64_t n, const Pred &pred) {
  if (!pred(0, top[tl.off[nlev - 1]])) return -1;
  int64_t s = 0;
#pragma unroll
  for (int L = kMaxLevels - 1; L >= 0; --L) {
    if (L < nlev && L >= tl.ltop) {
      const int64_t stride = int64_t(1) << (3 * L);
      const int64_t cnt = (n + stride - 1) / stride;
      const int64_t base = s * 8;
      const RPhi *blk = top + tl.off[L] + base;
      int c = 0;
#pragma unroll
      for (int q = 1; q < 8; ++q)
        if (base + q < cnt && pred((base + q) * stride, blk[q])) c = q;
      s = base + c;
    }
  }
  return static_cast<int32_t>(s);
}

// Star outputs: the staged record, its radix key and c = the number of old
// radii <= rn, or the state arrays in place.  c is monotone in rn, so the
// step's sort groups stars by c before it compares radii; escapers and
// non-finite radii are marked kBucketEsc and dropped.
template <bool TO_STAGE, typename MT>
__device__ __forceinline__ void emit(int64_t i, double rn, double vrn, double vtn, MT mi,
                                     uint32_t sid, int64_t c, double *__restrict__ r_new,
                                     double *__restrict__ vr, double *__restrict__ vt,
                                     StageRec<MT> *__restrict__ stage,
                                     uint64_t *__restrict__ keys, uint32_t *__restrict__ bkey) {
  if (TO_STAGE) {
    StageRec<MT> rec{};
    rec.r = rn;
    rec.vr = vrn;
    rec.vt = vtn;
    rec.m = mi;
    rec.id = sid;
    stage[i] = rec;
    const uint64_t key = rbits(rn);
    keys[i] = key;
    bkey[i] = key < 0x7FF0000000000000ull ? static_cast<uint32_t>(c) : kBucketEsc;
  } else {
    r_new[i] = rn;
    vr[i] = vrn;
    vt[i] = vtn;
  }
}

// New velocity from Q at the new radius: J conserved, E conserved in the old
// potential, the sign of v_r from the top bit of the sign draw's first word.
__device__ __forceinline__ void finish(double rn, double qn, double J, double J2,
                                       uint32_t sign_word, double &vrn, double &vtn,
                                       uint32_t &fl) {
  const double vmag = sqrt(qn > 0.0 ? qn : 0.0);
  vrn = (sign_word >> 31) ? -vmag : vmag;
  vtn = (J2 == 0.0) ? 0.0 : J / rn;
  if (!isfinite(rn) || !isfinite(vrn) || !isfinite(vtn)) fl |= CMC_ST_NONFINITE;
}

__device__ __forceinline__ void or_status(cmc_scalars *sc, uint32_t fl) {
  if (__ballot(fl != 0)) {
    uint32_t wf = fl;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wf |= __shfl_xor(wf, o, 64);
    if ((threadIdx.x & 63) == 0 && wf) atomicOr(&sc->status, wf);
  }
}

// The star's LFSR113 state after its draws: staged for the sort, or in place.
template <bool TO_STAGE>
__device__ __forceinline__ void put_lfsr(const ClusterArgs &A, int64_t i, const Lfsr &g) {
  if (TO_STAGE)
    A.w.rng_stage[i] = g;
  else
    store_lfsr(A.s.rng, i, g);
}

template <class Ctx, typename MT, bool TO_STAGE, bool LF>
__global__ __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(4)))
void k_orbit_bracket(Ctx ctx, uint32_t step_arg, double bound_factor, int corr) {
  extern __shared__ RPhi top[];
  __shared__ double shd[BT / 64];
  __shared__ GParams prm[2 * BT];
  const ClusterArgs &A = ctx.args();
  const uint32_t step = step_of(A, step_arg);
  const Levels lv = levels_of(A.w);
  const OrbitTop &tl = A.top;
  const RIndex ix{A.s.r, A.w.rx_start, A.w.rx_ctl};
  const MS *__restrict__ ms = A.w.ms;
  const MT *__restrict__ m = static_cast<const MT *>(A.s.m);
  double *__restrict__ vr = A.s.vr;
  double *__restrict__ vt = A.s.vt;
  const uint32_t *__restrict__ id = A.s.id;
  double *__restrict__ r_new = A.s.r_new;
  StageRec<MT> *__restrict__ stage = static_cast<StageRec<MT> *>(A.w.stage);
  uint64_t *__restrict__ keys = A.w.keys[0];
  uint32_t *__restrict__ bkey = A.w.bkey;
  OrbitRec *__restrict__ orec = A.w.orec;
  RPhi *__restrict__ cor = A.w.cor;
  double *__restrict__ pn = A.w.pn;
  cmc_scalars *__restrict__ sc = A.s.sc;
  double *__restrict__ part = A.w.red_part;
  const uint64_t seed = A.seed;
  const RIndexCtl ictl = *ix.ctl;
  const int64_t n = ictl.n;
  const RPhi *tab = lv.lev[0];
  GParams *wprm = prm + (threadIdx.x & ~63);
  for (int L = tl.ltop; L < lv.nlev; ++L)
    for (int e = threadIdx.x; e < tl.len[L]; e += BT) top[tl.off[L] + e] = lv.lev[L][e];
  __syncthreads();

  double c_esc = 0.0, e_esc = 0.0;
  uint32_t fl = 0;
  const int64_t tiles = (n + BT - 1) / BT;
  const int64_t blk = ctx.block(), nblk = ctx.nblocks();
  for (int64_t tile = blk; tile < tiles; tile += nblk) {  // block-uniform
    const int64_t i = tile * BT + threadIdx.x;
    double E = 0.0, J = 0.0, J2 = 0.0, vri = 0.0, vti = 0.0;
    if (i < n) {
      const RPhi me = tab[i];
      if (corr) cor[i] = me;  // r_old and Phi_old(r_old)
      // an LFSR113 state moves with its star; a Philox step stages it as it
      // is (an LFSR step stages it after the star's draws, and every kept
      // star draws at least its sign)
      if (TO_STAGE && !LF && A.s.rng) A.w.rng_stage[i] = load_lfsr(A.s.rng, i);
      vri = vr[i];
      vti = vt[i];
      E = me.phi + 0.5 * (vri * vri + vti * vti);
      J = me.r * vti;
      J2 = J * J;
    }
    const bool bound = i < n && E < 0.0;
    const int32_t ii = static_cast<int32_t>(i);
    // brackets: the LDS levels per lane, the rest by groups of 8 lanes
    int32_t t0 = -1, t1 = -1;
    if (bound) {
      t0 = top_descend(top, tl, lv.nlev, n, QNeg{2.0 * E, J2, ii});
      t1 = top_descend(top, tl, lv.nlev, n, QNonNeg{2.0 * E, J2, ii});
    }
    int64_t kmin_g, kmax_g;
    group_descend2<GQNeg, GQNonNeg>(lv, tl.ltop, n, GParams{2.0 * E, J2, ii, t0},
                                    GParams{2.0 * E, J2, ii, t1}, wprm, wprm + BT, kmin_g,
                                    kmax_g);

    if (i < n) {
      OrbitRec rec{E, J, 0.0, 0.0, -1.0, 0, 0};
      if (!(E < 0.0)) {  // unbound: leaves the cluster
        c_esc += 1.0;
        e_esc += load_mass(m, i) * E;
        fl |= CMC_ST_ESCAPER;
        if (E != E) fl |= CMC_ST_NONFINITE;
        emit<TO_STAGE>(i, kInf, vri, vti, m[i], id[i], 0, r_new, vr, vt, stage, keys, bkey);
      } else {
        const int64_t kmin = kmin_g, kmax = kmax_g;
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
        const double rc = 0.5 * (rmax + rmin), ra = 0.5 * (rmax - rmin);
        double F = -1.0;
        double rdone = rmin;  // radius of an orbit finished without trials
        if (ra > 0.0) {
          const double glo = (J2 != 0.0) ? sqrt(2.0 * ra / fabs(dq_in(ms, kmin, rmin, J2))) : 0.0;
          const double ghi = sqrt(2.0 * ra / fabs(dq_in(ms, kmax, rmax, J2)));
          F = bound_factor * (glo > ghi ? glo : ghi);
          if (!(F > 0.0 && F < kInf)) {
            F = -1.0;
            rdone = rc;
            fl |= CMC_ST_NUMERIC;
          }
        }
        if (F > 0.0) {
          rec.rmin = rmin;
          rec.rmax = rmax;
          rec.F = F;
          rec.kmin = static_cast<int32_t>(kmin);
          rec.kmax = static_cast<int32_t>(kmax);
        } else {
          const double rn = rdone + 0.0;
          const int64_t kn = interval_in(ix, ictl, rn, kmin, kmax);
          const double phn = phi_in(lv, ms, kn, rn);
          const double qn = 2.0 * E - 2.0 * phn - (J2 == 0.0 ? 0.0 : J2 / (rn * rn));
          if (corr) pn[i] = phn;
          U4 ws;
          if (LF) {
            Lfsr g = load_lfsr(A.s.rng, i);
            ws = lfsr_block(g);
            put_lfsr<TO_STAGE>(A, i, g);
          } else {
            ws = philox(id[i], step, kSign, 0u, seed);
          }
          double vrn, vtn;
          finish(rn, qn, J, J2, ws.x, vrn, vtn, fl);
          emit<TO_STAGE>(i, rn, vrn, vtn, m[i], id[i], rindex_last_le(ix, ictl, rn) + 1, r_new,
                         vr, vt, stage, keys, bkey);
        }
      }
      orec[i] = rec;
    }
  }
  or_status(sc, fl);
  c_esc = block_sum<BT>(c_esc, shd);
  e_esc = block_sum<BT>(e_esc, shd);
  if (threadIdx.x == 0) {
    part[2 * blk] = c_esc;
    part[2 * blk + 1] = e_esc;
  }
}

template <class Ctx, typename MT, bool TO_STAGE, bool MIXED, bool LF>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(5)))
void k_orbit_trials(Ctx ctx, uint32_t step_arg, int32_t trial_cap, int corr) {
  __shared__ double shd[NT / 64];
  const ClusterArgs &A = ctx.args();
  const uint32_t step = step_of(A, step_arg);
  const Levels lv = levels_of(A.w);
  const RIndex ix{A.s.r, A.w.rx_start, A.w.rx_ctl};
  const MS *__restrict__ ms = A.w.ms;
  const MT *__restrict__ m = static_cast<const MT *>(A.s.m);
  double *__restrict__ vr = A.s.vr;
  double *__restrict__ vt = A.s.vt;
  const uint32_t *__restrict__ id = A.s.id;
  double *__restrict__ r_new = A.s.r_new;
  StageRec<MT> *__restrict__ stage = static_cast<StageRec<MT> *>(A.w.stage);
  uint64_t *__restrict__ keys = A.w.keys[0];
  uint32_t *__restrict__ bkey = A.w.bkey;
  const OrbitRec *__restrict__ orec = A.w.orec;
  double *__restrict__ pn = A.w.pn;
  cmc_scalars *__restrict__ sc = A.s.sc;
  double *__restrict__ part = A.w.red_part + 2 * A.w.star_blocks;
  const uint64_t seed = A.seed;
  const RIndexCtl ictl = *ix.ctl;
  const int64_t n = ictl.n;
  const PhiBounds pb{A.w.phib, A.w.phib_ctl[0], static_cast<uint32_t>(A.w.phib_ctl[1]),
                     lv.lev[0][0].phi};
  const int64_t blk = ctx.block();
  const int lane = threadIdx.x & 63;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t wave = blk * (NT / 64) + (threadIdx.x >> 6);
  const int64_t c_end0 = (wave + 1) * kChunk;
  const int64_t c_end = c_end0 < n ? c_end0 : n;
  int64_t cursor = wave * kChunk;  // wave-uniform
  uint32_t c_tr = 0, c_viol = 0, c_cap = 0;
  uint32_t fl = 0;

  // lane state: current star and its orbit
  bool busy = false;
  int64_t i = 0;
  double E = 0.0, J = 0.0, J2 = 0.0, rc = 0.0, ra = 0.0, F = 0.0;
  int64_t kmin = 0, kmax = 0;
  uint32_t sid = 0;
  int32_t j = 0;
  double r0 = 0.0;
  Lfsr lg{};  // the star's LFSR113 stream (LF)

  for (;;) {
    // idle lanes take the chunk's next stars that still need trials
    for (;;) {
      const uint64_t need = __ballot(!busy);
      if (need == 0ull || cursor >= c_end) break;
      const int64_t mine = cursor + __popcll(need & lt);
      cursor += __popcll(need);
      if (!busy && mine < c_end) {
        const OrbitRec o = orec[mine];
        if (o.F > 0.0) {
          busy = true;
          i = mine;
          E = o.E;
          J = o.J;
          J2 = J * J;
          rc = 0.5 * (o.rmax + o.rmin);
          ra = 0.5 * (o.rmax - o.rmin);
          F = o.F;
          kmin = o.kmin;
          kmax = o.kmax;
          sid = id[mine];
          j = 0;
          if (LF) lg = load_lfsr(A.s.rng, mine);
        }
      }
    }
    if (__ballot(busy) == 0ull) break;
    // one rejection trial per busy lane; the interval search runs in groups
    double X2 = 0.0, cs = 0.0;
    if (busy) {
      const U4 w = LF ? lfsr_block(lg) : philox(sid, step, kOrbit, static_cast<uint32_t>(j), seed);
      if (MIXED) {
        // Trial angle and acceptance in FP32.  With s = pi (X - 1/2), the
        // offset of r from the nearer turning point is r_a (1 - |sin s|) =
        // 2 r_a sin^2(pi X' / 2), X' = min(X, 1 - X) (exact in FP32), and
        // cos s = sin(pi X'): both keep full relative precision near the
        // turning points, where rc + ra sin s in FP32 would round the offset
        // to a multiple of 2^-24 r_a.
        const float X = u01f(w.y);
        const bool upper = X > 0.5f;
        const float Xl = upper ? 1.0f - X : X;
        float hs, hc;
        sincosf(static_cast<float>(0.5 * kPi) * Xl, &hs, &hc);
        const double off = 2.0 * ra * static_cast<double>(hs * hs);
        r0 = upper ? (rc + ra) - off : (rc - ra) + off;
        cs = 2.0f * hs * hc;
        X2 = u01f(w.w);
      } else {
        const double X = u01(w.y, w.x);
        X2 = u01(w.w, w.z);
        const double s0 = kPi * (X - 0.5);
        double ss;
        sincos(s0, &ss, &cs);
        r0 = rc + ra * ss;
      }
      ++j;
      ++c_tr;
    }
    int64_t kg = 0;
    // a trial that is certainly rejected needs no interval (the capped last
    // trial always looks its interval up: its radius is kept)
    const bool settled =
        busy && j < trial_cap && surely_rejected<MIXED>(pb, r0, E, J2, ra, cs, F, X2);
    if (busy && !settled) {
      kg = rindex_last_le(ix, ictl, r0);
      const int64_t k0 = kg < kmin ? kmin : (kg > kmax ? kmax : kg);
      double phn = phi_in(lv, ms, k0, r0);
      const double q0 = 2.0 * E - 2.0 * phn - J2 / (r0 * r0);
      bool done = false;
      double qn = 0.0;
      if (q0 > 0.0) {
        bool over, acc;
        if (MIXED) {
          const float g0 = static_cast<float>(ra * cs) / sqrtf(static_cast<float>(q0));
          const float Ff = static_cast<float>(F);
          over = g0 > Ff;
          acc = Ff * static_cast<float>(X2) < g0;
        } else {
          const double g0 = ra * cs / sqrt(q0);
          over = g0 > F;
          acc = F * X2 < g0;
        }
        if (over) {
          ++c_viol;
          fl |= CMC_ST_BOUND;
        }
        if (acc) {
          done = true;
          qn = q0;
        }
      }
      if (!done && j >= trial_cap) {  // give up: keep the last trial radius
        done = true;
        ++c_cap;
        fl |= CMC_ST_TRIAL_CAP;
        const double rn = r0 + 0.0;
        const int64_t kn = interval_in(ix, ictl, rn, kmin, kmax);
        phn = phi_in(lv, ms, kn, rn);
        qn = 2.0 * E - 2.0 * phn - (J2 == 0.0 ? 0.0 : J2 / (rn * rn));
      }
      if (done) {
        const double rn = r0 + 0.0;
        if (corr) pn[i] = phn;  // Phi_old(r_new)
        const U4 ws = LF ? lfsr_block(lg) : philox(sid, step, kSign, 0u, seed);
        if (LF) put_lfsr<TO_STAGE>(A, i, lg);
        double vrn, vtn;
        finish(rn, qn, J, J2, ws.x, vrn, vtn, fl);
        emit<TO_STAGE>(i, rn, vrn, vtn, m[i], sid, kg + 1, r_new, vr, vt, stage, keys, bkey);
        busy = false;
      }
    }
  }
  or_status(sc, fl);
  const double t_tr = block_sum<NT>(static_cast<double>(c_tr), shd);
  const double t_viol = block_sum<NT>(static_cast<double>(c_viol), shd);
  const double t_cap = block_sum<NT>(static_cast<double>(c_cap), shd);
  if (threadIdx.x == 0) {
    double *pp = part + 3 * blk;
    pp[0] = t_tr;
    pp[1] = t_viol;
    pp[2] = t_cap;
  }
}

// The potential at the bound table's edges (after the radial index is built),
// grid-stride over the edges.
template <class Ctx>
__global__ __launch_bounds__(NT) void k_phi_bounds(Ctx ctx) {
  const ClusterArgs &A = ctx.args();
  const RIndex ix{A.s.r, A.w.rx_start, A.w.rx_ctl};
  const RIndexCtl ictl = *ix.ctl;
  if (ictl.n == 0) return;
  const Levels lv = levels_of(A.w);
  uint32_t shift = 0;
  while (((ictl.hi - ictl.lo) >> shift) >= static_cast<uint64_t>(kPhiBins)) ++shift;
  for (int64_t j = ctx.block() * NT + threadIdx.x; j <= kPhiBins; j += ctx.nblocks() * NT) {
    uint64_t bits = ictl.lo + (static_cast<uint64_t>(j) << shift);
    bits = bits < 0x7FF0000000000000ull ? bits : 0x7FF0000000000000ull;
    const double x = __builtin_bit_cast(double, bits);
    A.w.phib[j] = phi_in(lv, A.w.ms, rindex_last_le(ix, ictl, x), x);
  }
  if (ctx.block() == 0 && threadIdx.x == 0) {
    A.w.phib_ctl[0] = ictl.lo;
    A.w.phib_ctl[1] = shift;
  }
}

constexpr int FT = 1024;

// One block per cluster: the cluster's bracket and trial partials.
template <class Ctx>
__global__ __launch_bounds__(FT) void k_orbit_sum(Ctx ctx) {
  __shared__ double sh[FT / 64];
  const ClusterArgs &A = ctx.args();
  const double *__restrict__ pa = A.w.red_part;
  const double *__restrict__ pb = A.w.red_part + 2 * A.w.star_blocks;
  const int64_t na = A.bracket_blocks;
  const int64_t nb = blocks_of(kShTrials, A.w, A.s.cap);
  cmc_scalars *__restrict__ sc = A.s.sc;
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t b = threadIdx.x; b < na; b += FT) {
    v[0] += pa[2 * b];
    v[4] += pa[2 * b + 1];
  }
  for (int64_t b = threadIdx.x; b < nb; b += FT)
#pragma unroll
    for (int q = 0; q < 3; ++q) v[1 + q] += pb[3 * b + q];
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
template <class Ctx>
__global__ __launch_bounds__(NT) void k_table_pack(Ctx ctx) {
  const ClusterArgs &A = ctx.args();
  const int64_t k = ctx.block() * NT + threadIdx.x;
  if (k >= A.s.sc->n) return;
  put_table(levels_of(A.w), A.w.ms, k, A.s.r[k], A.s.phi[k], A.s.mcum[k], A.s.ssuf[k]);
}

template <class L, typename MT, bool TO_STAGE, bool LF>
hipError_t run2(const L &l, const cmc_params &p, int corr, hipStream_t st) {
  const int32_t cap = p.trial_cap > 0 ? p.trial_cap : 10000;
  const double bf = p.bound_factor > 0.0 ? p.bound_factor : 1.2;
  using Cb = decltype(l.ctx(kShBracket));
  using Ct = decltype(l.ctx(kShTrials));
  k_phi_bounds<<<l.grid(kShDiag), NT, 0, st>>>(l.ctx(kShDiag));
  k_orbit_bracket<Cb, MT, TO_STAGE, LF>
      <<<l.grid(kShBracket), BT, sizeof(RPhi) * l.top_entries(), st>>>(l.ctx(kShBracket), p.step,
                                                                       bf, corr);
  if (p.precision == CMC_MIXED)
    k_orbit_trials<Ct, MT, TO_STAGE, true, LF><<<l.grid(kShTrials), NT, 0, st>>>(
        l.ctx(kShTrials), p.step, cap, corr);
  else
    k_orbit_trials<Ct, MT, TO_STAGE, false, LF><<<l.grid(kShTrials), NT, 0, st>>>(
        l.ctx(kShTrials), p.step, cap, corr);
  k_orbit_sum<<<l.grid(kShOne), FT, 0, st>>>(l.ctx(kShOne));
  return hipGetLastError();
}

}  // namespace

static_assert(sizeof(OrbitRec) == 48, "orbit record layout");
static_assert(BT == kBracketThreads && kChunk == kTrialChunk, "launch shapes");

// Levels from the top down while they fit kTopBytes of LDS.
OrbitTop orbit_top(const Workspace &w, int64_t cap) {
  OrbitTop tl{};
  int64_t tot = 0;
  tl.ltop = w.nlev;
  for (int L = w.nlev - 1; L >= 0; --L) {
    const int64_t stride = int64_t(1) << (3 * L);
    const int64_t len = (cap + stride - 1) / stride;
    if ((tot + len) * static_cast<int64_t>(sizeof(RPhi)) > kTopBytes) break;
    tl.off[L] = static_cast<int32_t>(tot);
    tl.len[L] = static_cast<int32_t>(len);
    tot += len;
    tl.ltop = L;
  }
  tl.entries = static_cast<int32_t>(tot);
  return tl;
}

hipError_t launch_table_pack(const Target &t, hipStream_t st) {
  return dispatch(t, [&](const auto &l) {
    k_table_pack<<<l.grid(kShStar), NT, 0, st>>>(l.ctx(kShStar));
    return hipGetLastError();
  });
}

hipError_t launch_orbit(const Target &t, bool m_f32, const cmc_params &p, bool to_stage,
                        bool corr, bool rindex_ready, hipStream_t st) {
  if (!rindex_ready) {
    const hipError_t e = launch_rindex(t, st);
    if (e != hipSuccess) return e;
  }
  const int c = (to_stage && corr) ? 1 : 0;  // correction terms only for a staged step
  const bool lf = p.rng == CMC_RNG_LFSR113;
  return dispatch(t, [&](const auto &l) {
    using L = std::decay_t<decltype(l)>;
    if (lf) {
      if (m_f32)
        return to_stage ? run2<L, float, true, true>(l, p, c, st)
                        : run2<L, float, false, true>(l, p, c, st);
      return to_stage ? run2<L, double, true, true>(l, p, c, st)
                      : run2<L, double, false, true>(l, p, c, st);
    }
    if (m_f32)
      return to_stage ? run2<L, float, true, false>(l, p, c, st)
                      : run2<L, float, false, false>(l, p, c, st);
    return to_stage ? run2<L, double, true, false>(l, p, c, st)
                    : run2<L, double, false, false>(l, p, c, st);
  });
}

}  // namespace cmc

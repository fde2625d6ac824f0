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
// Brackets.  The lower and the upper bracket are each "the last index k
// where a predicate monotone in k holds".  They descend the sampled levels of
// the table (level L = every 8^L-th (r, Phi)): per level, the 8 children of
// the current sample are one aligned cache line, and the count of children
// that satisfy the predicate is the next sample.  The top levels (a few
// thousand entries) sit in LDS and each lane descends them alone; below
// them, lanes work in groups of 8 so that every node is one coalesced load.
// Brackets are unique, so this finds the index a bisection over the whole
// table finds.  Two forms, with the same result:
//  - direct (k_orbit_bracket): each star's wavefront searches its own two
//    brackets to the bottom; below the LDS top every level is a random line
//    of a table far larger than the L2.
//  - sorted (k_oq_*): the searches are first grouped by the LDS-level sample
//    they reached (a counting sort of 2 N small records), so that the
//    searches sharing a subtree run together: where the subtree is small
//    enough (4096 stars at most), a block holds it whole in LDS, level 0
//    and the (M, S) included, and its searches read no table line at all;
//    a deeper subtree is found in the L2.  Each search writes its half of
//    the star's orbit record where it sits in that order, and the trial
//    kernel finds the two halves there.
// Either way the roots inside the brackets and the rejection bound F follow.
// k_orbit_trials then draws the radii: each wavefront owns a chunk of stars
// and every lane draws trials for one star at a time, taking the chunk's
// next star as soon as its own is accepted, so the loop does not wait for
// the unluckiest lane of the wavefront.  The interval of a trial radius
// comes from the radial bucket index (rindex.hip); a trial that the
// potential-bound table proves rejected skips that lookup (see
// surely_rejected).
#include <algorithm>
#include <type_traits>

#include "cmc_internal.hpp"

namespace cmc {
namespace {

constexpr int NT = kBlock;
constexpr int BT = 512;         // threads per block of the bracket kernel
// group searches whose loads are in flight together: 4 keeps the bracket
// kernel at 86 VGPRs without spills (8 needs 118); its occupancy is set by
// the LDS-resident top levels either way, and 4 measured ~1 % faster
constexpr int kGroupBatch = 4;
static_assert(16 % kGroupBatch == 0, "batches split the 16 searches of a group");

// Sign of Q_k = 2E - 2Phi_k - J^2/r_k^2 without the division:
// (2E - 2Phi_k) r_k^2 against J^2.  A star at r_k = 0 takes the limit r -> 0:
// Q = -inf when J != 0 (the J^2/r^2 term wins, even against Phi_k = -inf),
// else 2E - 2Phi_k.
// (Both sides are evaluated and combined by select: lanes of a wavefront
// take them alike, with no branch.)
__device__ __forceinline__ bool q_neg(double twoE, double J2, const RPhi &e) {
  const double d = twoE - 2.0 * e.phi;
  const bool at0 = (J2 > 0.0) | (d < 0.0);
  const bool off0 = d * (e.r * e.r) < J2;
  return e.r == 0.0 ? at0 : off0;
}
__device__ __forceinline__ bool q_nonneg(double twoE, double J2, const RPhi &e) {
  const double d = twoE - 2.0 * e.phi;
  const bool at0 = (J2 == 0.0) & (d >= 0.0);
  const bool off0 = d * (e.r * e.r) >= J2;
  return e.r == 0.0 ? at0 : off0;
}
// Potential inside interval k from the defining sum: -(M_k / x + S_k); flat
// at Phi_0 inside the innermost star.
__device__ __forceinline__ double phi_in(const Levels &lv, const MS *__restrict__ ms, int64_t k,
                                         double x) {
  if (k < 0) return lv.lev[0][0].phi;
  const MS t = ms[k];
  return -(t.M / x + t.S);
}

// dQ/dr at x in interval k (M = M_k; no mass inside the innermost star)
__device__ __forceinline__ double dq_of(double M, int64_t k, double x, double J2) {
  const double grav = (k >= 0) ? -2.0 * M / (x * x) : 0.0;
  return grav + 2.0 * J2 / (x * x * x);
}
__device__ __forceinline__ double dq_in(const MS *__restrict__ ms, int64_t k, double x,
                                        double J2) {
  return dq_of(k >= 0 ? ms[k].M : 0.0, k, x, J2);
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

// ---------------------------------------------------------------- LDS levels
// Each lane descends the LDS-resident levels alone: per level, the 7 other
// children of its sample, one 16-byte read each (the padded layout spreads
// the lanes' nodes over the banks).  Q_k < 0 and k < below: the lower
// bracket; Q_k >= 0 or k <= upto: the upper one.
struct QNeg {
  double twoE, J2;
  int32_t below;
  __device__ bool operator()(int32_t k, const RPhi &e) const {
    const bool in = k < below;
    const bool q = q_neg(twoE, J2, e);
    return in & q;
  }
};
struct QNonNeg {
  double twoE, J2;
  int32_t upto;
  __device__ bool operator()(int32_t k, const RPhi &e) const {
    const bool in = k <= upto;
    const bool q = q_nonneg(twoE, J2, e);
    return in | q;
  }
};
// Either bracket for the search kernel: c >= 0 the lower bracket below star
// c, c < 0 the upper bracket of star -c - 1.
struct QAny {
  double twoE, J2;
  int32_t c;
  __device__ bool operator()(int32_t k, const RPhi &e) const {
    const bool low = (k < c) & q_neg(twoE, J2, e);
    const bool up = (k <= -c - 1) | q_nonneg(twoE, J2, e);
    return c >= 0 ? low : up;
  }
};

// The same predicates for the staged search, evaluated without branches:
// lower (hi false) Q_k < 0 and k < lim, upper Q_k >= 0 or k <= lim (lim =
// the star's index).  The sign tests are q_neg's and q_nonneg's.
struct QSel {
  double twoE, J2;
  int32_t lim;
  bool hi;
};
__device__ __forceinline__ bool qsel(const QSel &p, int32_t k, const RPhi &e) {
  const double d = p.twoE - 2.0 * e.phi;
  const double w = d * (e.r * e.r);
  const bool r0 = e.r == 0.0;
  const bool neg0 = (p.J2 > 0.0) | (d < 0.0), negw = w < p.J2;
  const bool non0 = (p.J2 == 0.0) & (d >= 0.0), nonw = w >= p.J2;
  const bool neg = r0 ? neg0 : negw;
  const bool nonneg = r0 ? non0 : nonw;
  const bool up = (k <= p.lim) | nonneg;
  const bool low = (k < p.lim) & neg;
  return p.hi ? up : low;
}

// LDS slot of entry e of a padded level that starts at slot off.
__device__ __forceinline__ int64_t pad_slot(int64_t off, int64_t e) { return off + e + (e >> 3); }

// The levels [ltop, nlev) -- at most kTopEntries slots, see top_levels() --
// are copied into LDS by every block of the kernels that start the searches.
__device__ __forceinline__ void load_top(RPhi *top, const Levels &lv, const OrbitTop &tl,
                                         int nthreads) {
  for (int L = tl.ltop; L < lv.nlev; ++L)
    for (int e = threadIdx.x; e < tl.len[L]; e += nthreads)
      top[pad_slot(tl.off[L], e)] = lv.lev[L][e];
}

// Descent of the LDS levels: the sample of level ltop below which the last
// index satisfying pred lies (-1: no index does).  With ltop = 0 that is the
// index itself.
// The last child c in 0..7 of a node (entries blk[0..7], child 0 known to
// hold) where pred holds, by bisection over the 8: the predicate is monotone
// in the index, so 3 evaluations find it.  Children from `avail` on do not
// exist (they count as not holding).  k0 + q * stride: child q's index.
template <class Pred>
__device__ __forceinline__ int node_last(const RPhi *blk, int avail, int32_t k0, int32_t stride,
                                         const Pred &pred) {
  int c = 0;
#pragma unroll
  for (int h = 4; h >= 1; h >>= 1) {
    const int q = c + h;
    const RPhi e = blk[q < avail ? q : avail - 1];  // a child that exists
    const bool ok = (q < avail) & pred(k0 + q * stride, e);
    c = ok ? q : c;
  }
  return c;
}

// node_last for qsel, reading all probed children (the caller's node lies
// wholly inside its LDS array) and choosing by select.
__device__ __forceinline__ int node_last_sel(const RPhi *blk, int avail, int32_t k0,
                                             int32_t stride, const QSel &p) {
  int c = 0;
#pragma unroll
  for (int h = 4; h >= 1; h >>= 1) {
    const int q = c + h;
    const RPhi e = blk[q];
    const bool ok = (q < avail) & qsel(p, k0 + q * stride, e);
    c = ok ? q : c;
  }
  return c;
}

template <class Pred>
__device__ __forceinline__ int32_t top_descend(const RPhi *top, const OrbitTop &tl, int nlev,
                                               int64_t n, const Pred &pred) {
  if (!pred(0, top[tl.off[nlev - 1]])) return -1;
  int32_t s = 0;
#pragma unroll
  for (int L = kMaxLevels - 1; L >= 0; --L) {
    if (L < nlev && L >= tl.ltop) {
      const int32_t stride = int32_t(1) << (3 * L);
      const int32_t cnt = static_cast<int32_t>((n + stride - 1) >> (3 * L));
      const int32_t base = s * 8;
      const RPhi *blk = top + pad_slot(tl.off[L], base);
      s = base + node_last(blk, cnt - base, base * stride, stride, pred);
    }
  }
  return s;
}

// ---------------------------------------------------------------- group search
// Below the LDS levels the searches run cooperatively: lanes form groups of 8
// (group g = lanes 8g..8g+7), and each group runs the searches of its 8
// lanes together.  Per level, lane q loads child q of each current sample,
// so every node is one coalesced 128-byte load instead of 8 loads per lane,
// and a ballot counts the children that satisfy the predicate.  Predicate
// parameters travel through LDS.  Every lane of the wavefront must call it.
struct GParams {
  double a, b;  // 2E, J^2
  int32_t c;    // the star's index: below (lower bracket) or upto (upper); see GQAny
  int32_t s0;   // the sample the search starts below (-1: no index holds)
};
struct GQNeg {
  __device__ static bool eval(const GParams &p, int64_t k, const RPhi &e) {
    const bool in = k < p.c;
    return in & q_neg(p.a, p.b, e);
  }
};
struct GQNonNeg {
  __device__ static bool eval(const GParams &p, int64_t k, const RPhi &e) {
    const bool in = k <= p.c;
    return in | q_nonneg(p.a, p.b, e);
  }
};
// Either bracket: c >= 0 is the lower bracket below star c, c < 0 the upper
// bracket of star -c - 1.
struct GQAny {
  __device__ static bool eval(const GParams &p, int64_t k, const RPhi &e) {
    const bool low = (k < p.c) & q_neg(p.a, p.b, e);
    const bool up = (k <= -static_cast<int64_t>(p.c) - 1) | q_nonneg(p.a, p.b, e);
    return p.c >= 0 ? low : up;
  }
};

// Descent of the levels below lhi + 1 down to level 0 for two searches per
// lane (predicates PA and PB), each starting below the sample s0 of level
// lhi + 1 that its lane brings (-1: no index holds).  The loads of
// kGroupBatch searches are in flight together.
template <class PA, class PB>
__device__ __forceinline__ void group_descend2(const Levels &lv, int lhi, int64_t n,
                                               const GParams &ma, const GParams &mb,
                                               GParams *prm_a, GParams *prm_b, int32_t &ka,
                                               int32_t &kb) {
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
    if (L <= lhi) {
      // re-read the parameters from LDS at every level rather than keep
      // 16 sets of them live in registers
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      const int64_t stride = int64_t(1) << (3 * L);
      const int64_t cnt = (n + stride - 1) >> (3 * L);
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

// One search per lane, the same way (8 per group, all 8 loads of a level in
// flight), from below sample mine.s0 of level lhi + 1 to level 0; returns
// the lane's own result.
template <class P>
__device__ __forceinline__ int32_t group_descend1(const Levels &lv, int lhi, int64_t n,
                                                  const GParams &mine, GParams *wprm) {
  const int lane = threadIdx.x & 63, g = lane >> 3, q = lane & 7;
  wprm[lane] = mine;
  __builtin_amdgcn_wave_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  int32_t s[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) s[u] = wprm[(g << 3) + u].s0;
#pragma unroll
  for (int L = kMaxLevels - 1; L >= 0; --L) {
    if (L <= lhi) {
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      const int64_t stride = int64_t(1) << (3 * L);
      const int64_t cnt = (n + stride - 1) >> (3 * L);
      const RPhi *lev = lv.lev[L];
      RPhi e[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t child = static_cast<int64_t>(s[u]) * 8 + q;
        e[u] = (s[u] >= 0 && child < cnt) ? lev[child] : RPhi{0.0, 0.0};
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const GParams p = wprm[(g << 3) + u];
        const int64_t child = static_cast<int64_t>(s[u]) * 8 + q;
        const bool ok = s[u] >= 0 && child < cnt && P::eval(p, child * stride, e[u]);
        const uint64_t m = __ballot(ok);
        const int c = __popcll((m >> (g << 3)) & 0xFFull);
        if (s[u] >= 0) s[u] = s[u] * 8 + c - 1;
      }
    }
  }
  __builtin_amdgcn_wave_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  int32_t r = s[0];
#pragma unroll
  for (int u = 1; u < 8; ++u)
    if (q == u) r = s[u];
  return r;
}

// ---------------------------------------------------------------- turning points
// The lower turning point in interval kmin (-1: inside the innermost star,
// where the potential is flat), from r^2 Q = 2(E + S_k) r^2 + 2 M_k r - J^2
// in the cancellation-free form, kept inside the interval [rl, rh]; with
// dQ/dr there.  t = (M, S) of the interval, phi0 = Phi_0 (used for kmin < 0).
// The root of r^2 Q in an interval [rl, rh] with (M, S) = t: with
// a = 2(E + S), b = 2M and s = b + sqrt(b^2 + 4 a J^2), the lower one is
// 2 J^2 / s (no cancellation), the upper one s / (-2a); where the root does
// not exist (s <= 0, a >= 0) the interval's inner or outer end.  hi selects
// the upper root; both forms of the search share this arithmetic.
__device__ __forceinline__ double interval_root(bool hi, MS t, double rl, double rh, double E,
                                                double J2) {
  const double a = 2.0 * (E + t.S);
  const double b = 2.0 * t.M;
  const double disc = b * b + 4.0 * a * J2;
  const double bs = b + sqrt(disc > 0.0 ? disc : 0.0);
  const double num = hi ? bs : 2.0 * J2;
  const double den = hi ? -2.0 * a : bs;
  const bool ok = hi ? (a < 0.0) : (den > 0.0);
  const double x = num / den;
  return ok ? x : (hi ? rh : rl);
}
__device__ __forceinline__ OrbitLo lower_point(int64_t kmin, MS t, double rl, double rh,
                                               double phi0, double E, double J, double J2) {
  double rmin;
  if (J2 == 0.0) {
    rmin = 0.0;
  } else if (kmin < 0) {
    rmin = J / sqrt(2.0 * (E - phi0));
  } else {
    rmin = interval_root(false, t, rl, rh, E, J2);
  }
  rmin = rmin < rl ? rl : (rmin > rh ? rh : rmin);
  OrbitLo o{};
  o.E = E;
  o.rmin = rmin;
  o.dq = (J2 != 0.0) ? dq_of(t.M, kmin, rmin, J2) : 0.0;
  o.kmin = static_cast<int32_t>(kmin);
  return o;
}
__device__ __forceinline__ OrbitLo finalize_lo(const RPhi *__restrict__ tab,
                                               const MS *__restrict__ ms, int64_t kmin, double E,
                                               double J, double J2) {
  const MS t = kmin >= 0 ? ms[kmin] : MS{0.0, 0.0};
  const double rl = kmin >= 0 ? tab[kmin].r : 0.0;
  const double phi0 = kmin < 0 ? tab[0].phi : 0.0;
  return lower_point(kmin, t, rl, tab[kmin + 1].r, phi0, E, J, J2);
}

// The upper turning point in interval kmax (n - 1: beyond the last star,
// rh = +inf), kept inside [rl, rh].
__device__ __forceinline__ OrbitHi upper_point(int64_t kmax, MS t, double rl, double rh,
                                               double E, double J, double J2) {
  double rmax = interval_root(true, t, rl, rh, E, J2);
  rmax = rmax < rl ? rl : (rmax > rh ? rh : rmax);
  OrbitHi o{};
  o.J = J;
  o.rmax = rmax;
  o.dq = dq_of(t.M, kmax, rmax, J2);
  o.kmax = static_cast<int32_t>(kmax);
  return o;
}
__device__ __forceinline__ OrbitHi finalize_hi(const RPhi *__restrict__ tab,
                                               const MS *__restrict__ ms, int64_t n, int64_t kmax,
                                               double E, double J, double J2) {
  const double rh = (kmax + 1 < n) ? tab[kmax + 1].r : kInf;
  return upper_point(kmax, ms[kmax], tab[kmax].r, rh, E, J, J2);
}

// The record of a star that leaves the cluster (E >= 0 or NaN): the trial
// kernel skips it.
__device__ __forceinline__ OrbitLo escaper_lo(double E) {
  OrbitLo o{};
  o.E = E;
  o.kmin = -1;
  return o;
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


// Per-star work of the pass before the searches: the energy-correction
// record, the staged RNG state, E and J, and the escapers (sent out here,
// their masses and energies summed; mark: note the escaper in its orbit
// record, where the records are in star order).  Returns whether the star
// is bound.
template <typename MT, bool TO_STAGE, bool LF>
__device__ __forceinline__ bool star_start(const ClusterArgs &A, int64_t i, int corr, double &E,
                                           double &J, double &J2, double &c_esc, double &e_esc,
                                           uint32_t &fl, bool mark) {
  const RPhi me = A.w.lev[0][i];
  if (corr) A.w.cor[i] = me;  // r_old and Phi_old(r_old)
  // an LFSR113 state moves with its star; a Philox step stages it as it is
  // (an LFSR step stages it after the star's draws, and every kept star
  // draws at least its sign)
  if (TO_STAGE && !LF && A.s.rng) A.w.rng_stage[i] = load_lfsr(A.s.rng, i);
  const double vri = A.s.vr[i], vti = A.s.vt[i];
  E = me.phi + 0.5 * (vri * vri + vti * vti);
  J = me.r * vti;
  J2 = J * J;
  if (E < 0.0) return true;
  // unbound: leaves the cluster
  const MT *__restrict__ m = static_cast<const MT *>(A.s.m);
  c_esc += 1.0;
  e_esc += load_mass(m, i) * E;
  fl |= CMC_ST_ESCAPER;
  if (E != E) fl |= CMC_ST_NONFINITE;
  emit<TO_STAGE>(i, kInf, vri, vti, m[i], A.s.id[i], 0, A.s.r_new, A.s.vr, A.s.vt,
                 static_cast<StageRec<MT> *>(A.w.stage), A.w.keys[0], A.w.bkey);
  if (mark) A.w.orec[i].lo = escaper_lo(E);
  return false;
}

// The escaper partials (count, sum of m E) of 512 stars at part[2 tile]:
// both forms of the pass write them per 512 consecutive stars, so the sum
// does not depend on the form or its launch settings.
template <int NTH>
__device__ __forceinline__ void esc_partials(double c_esc, double e_esc, double *shd,
                                             double *part, int64_t blk) {
  c_esc = block_sum<NTH>(c_esc, shd);
  e_esc = block_sum<NTH>(e_esc, shd);
  if (threadIdx.x == 0) {
    part[2 * blk] = c_esc;
    part[2 * blk + 1] = e_esc;
  }
}

// Direct form: every bracket searched to the bottom by the star's own
// wavefront (the LDS levels per lane, the rest by groups of 8 lanes); its
// blocks stay resident and loop over tiles of stars.  For tables whose levels
// below the LDS top are few or small.
template <class Ctx, typename MT, bool TO_STAGE, bool LF>
__global__ __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(4)))
void k_orbit_bracket(Ctx ctx, int corr) {
  extern __shared__ RPhi top[];
  __shared__ double shd[BT / 64];
  __shared__ GParams prm[2 * BT];
  const ClusterArgs &A = ctx.args();
  const Levels lv = levels_of(A.w);
  const OrbitTop &tl = A.top;
  const MS *__restrict__ ms = A.w.ms;
  OrbitRec *__restrict__ orec = A.w.orec;
  const RIndexCtl ictl = *A.w.rx_ctl;
  const int64_t n = ictl.n;
  const RPhi *tab = lv.lev[0];
  GParams *wprm = prm + (threadIdx.x & ~63);
  load_top(top, lv, tl, BT);
  __syncthreads();

  uint32_t fl = 0;
  const int64_t tiles = (n + BT - 1) / BT;
  const int64_t blk = ctx.block(), nblk = ctx.nblocks();
  for (int64_t tile = blk; tile < tiles; tile += nblk) {  // block-uniform
    const int64_t i = tile * BT + threadIdx.x;
    double c_esc = 0.0, e_esc = 0.0;
    double E = 0.0, J = 0.0, J2 = 0.0;
    const bool bound =
        i < n && star_start<MT, TO_STAGE, LF>(A, i, corr, E, J, J2, c_esc, e_esc, fl, true);
    const int32_t ii = static_cast<int32_t>(i);
    // brackets: the LDS levels per lane, the rest by groups of 8 lanes
    int32_t t0 = -1, t1 = -1;
    if (bound) {
      t0 = top_descend(top, tl, lv.nlev, n, QNeg{2.0 * E, J2, ii});
      t1 = top_descend(top, tl, lv.nlev, n, QNonNeg{2.0 * E, J2, ii});
    }
    int32_t kmin, kmax;
    group_descend2<GQNeg, GQNonNeg>(lv, tl.ltop - 1, n, GParams{2.0 * E, J2, ii, t0},
                                    GParams{2.0 * E, J2, ii, t1}, wprm, wprm + BT, kmin, kmax);
    if (bound) {
      orec[i].lo = finalize_lo(tab, ms, kmin, E, J, J2);
      orec[i].hi = finalize_hi(tab, ms, n, kmax, E, J, J2);
    }
    esc_partials<BT>(c_esc, e_esc, shd, A.w.red_part, tile);
  }
  or_status(A.s.sc, fl);
}

// ---------------------------------------------------------------- sorted searches
// The sorted form.  Below the LDS top every search costs a few random lines
// of a table far larger than the L2; grouped by the top-level sample it
// reached, the searches that share a subtree run together and find it in
// the L2.  k_oq_hist counts each tile's searches per sample, k_oq_colscan
// and k_oq_start turn the counts into offsets, k_oq_scatter sends every
// star's searches (E, J, index, sample) to their groups and finishes what
// needs no search, and k_oq_search runs the grouped searches.  Each search
// writes its half-record where it sits in the grouped order, coalesced; the
// scatter records the two places of every star (oq_pos), where the trial
// kernel reads them.  The lower turning points that the LDS levels already
// finish (interval -1) take a group of their own, after the samples', which
// no search block visits.  Brackets are unique, so the result is the one of
// the direct form.
constexpr int QT = 512;   // threads of the tile kernels
constexpr int CT = 1024;  // threads of the column scan
constexpr int QS = kQuerySearchBlock;
constexpr int kSubEntries = 704;  // LDS slots of a group's subtree in the search

// Samples of level ltop over the n stars (the groups of this pass).
__device__ __forceinline__ int64_t query_bins(const OrbitTop &tl, int64_t n) {
  return tl.ltop > 0 ? cdiv(n, int64_t(1) << (3 * tl.ltop)) : 0;
}

// Consecutive tiles (and search blocks) on one XCD: blocks go round-robin
// over the 8 XCDs, so logical tile (b mod 8) q + b / 8 puts each XCD on a
// contiguous eighth.
__device__ __forceinline__ int64_t xcd_order(int64_t b, int64_t nb) {
  const int64_t q = nb / 8;
  return b < 8 * q ? (b % 8) * q + b / 8 : b;
}

template <class Ctx>
__global__ __launch_bounds__(QT) void k_oq_hist(Ctx ctx) {
  extern __shared__ RPhi top[];
  __shared__ uint32_t hist[kTopEntries];
  const ClusterArgs &A = ctx.args();
  const OrbitTop &tl = A.top;
  const RIndexCtl ictl = *A.w.rx_ctl;
  const int64_t n = ictl.n;
  const int64_t bins = query_bins(tl, n);
  const int64_t t = ctx.block();
  const int64_t k0 = t * kQueryTile;
  if (bins == 0 || k0 >= n) return;  // block-uniform
  const Levels lv = levels_of(A.w);
  const RPhi *__restrict__ tab = lv.lev[0];
  uint32_t *__restrict__ node = A.w.oq_node;
  load_top(top, lv, tl, QT);
  for (int b = threadIdx.x; b <= bins; b += QT) hist[b] = 0u;
  __syncthreads();
  const int64_t k1 = k0 + kQueryTile < n ? k0 + kQueryTile : n;
  // two stars per thread and pass: four independent descents in flight
  for (int64_t i0 = k0 + threadIdx.x; i0 < k1; i0 += 2 * QT) {
    double E[2], J2[2];
    bool in[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int64_t i = i0 + u * QT;
      in[u] = i < k1;
      const int64_t ic = in[u] ? i : i0;
      const RPhi me = tab[ic];
      const double vri = A.s.vr[ic], vti = A.s.vt[ic];
      E[u] = me.phi + 0.5 * (vri * vri + vti * vti);
      const double J = me.r * vti;
      J2[u] = J * J;
    }
    int32_t t0[2], t1[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int32_t ii = static_cast<int32_t>(i0 + u * QT);
      t0[u] = top_descend(top, tl, lv.nlev, n, QNeg{2.0 * E[u], J2[u], ii});
      t1[u] = top_descend(top, tl, lv.nlev, n, QNonNeg{2.0 * E[u], J2[u], ii});
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (!in[u]) continue;
      // the two samples for the scatter: (t0 + 1) | t1 << 16, or none
      uint32_t code = 0xFFFFFFFFu;
      if (E[u] < 0.0) {
        atomicAdd(&hist[t0[u] >= 0 ? t0[u] : static_cast<int32_t>(bins)], 1u);
        atomicAdd(&hist[t1[u]], 1u);
        code = static_cast<uint32_t>(t0[u] + 1) | (static_cast<uint32_t>(t1[u]) << 16);
      }
      node[i0 + u * QT] = code;
    }
  }
  __syncthreads();
  uint32_t *__restrict__ row = A.w.oq_cnt + t * A.w.oq_bins;
  for (int b = threadIdx.x; b <= bins; b += QT) row[b] = hist[b];
}

// Block g: samples kQColGroup g .. kQColGroup (g + 1) - 1.  Counts become tile
// offsets inside the sample's group; oq_tot gets the group sizes.
template <class Ctx>
__global__ __launch_bounds__(CT) void k_oq_colscan(Ctx ctx) {
  const ClusterArgs &A = ctx.args();
  const int64_t n = A.w.rx_ctl->n;
  const int64_t bins = query_bins(A.top, n);
  // neighbouring column groups on one XCD: they share the count rows' lines
  const int64_t c0 = xcd_order(ctx.block(), ctx.nblocks()) * kQColGroup;
  if (bins == 0 || c0 > bins) return;  // block-uniform
  column_scan<CT, kQColGroup>(A.w.oq_cnt, A.w.oq_bins, cdiv(n, kQueryTile), c0, bins + 1,
                              A.w.oq_tot);
}

// One block per cluster: the first search of each group (oq_start[bins] is
// the number of searches), and the first block of the search kernel that
// works on each group, kQuerySearchChunk searches per block, or kStagedChunk
// where the subtree is staged whole (oq_chunk[bins] is the number of blocks
// with work).
template <class Ctx>
__global__ __launch_bounds__(QT) void k_oq_start(Ctx ctx) {
  __shared__ uint32_t sh[QT / 64];
  const ClusterArgs &A = ctx.args();
  const int64_t bins = query_bins(A.top, A.w.rx_ctl->n);
  const uint32_t *__restrict__ tot = A.w.oq_tot;
  uint32_t *__restrict__ start = A.w.oq_start;
  uint32_t *__restrict__ chunk = A.w.oq_chunk;
  uint32_t *__restrict__ bmap = A.w.oq_bmap;
  // groups: the bins samples' and the finished lower turning points' (no
  // search block)
  const int64_t groups = bins > 0 ? bins + 1 : 0;
  const uint32_t per = A.w.oq_staged ? kStagedChunk : kQuerySearchChunk;
  uint32_t carry = 0u, ccarry = 0u;
  for (int64_t b0 = 0; b0 < groups; b0 += QT) {
    const int64_t b = b0 + threadIdx.x;
    const uint32_t v = b < groups ? tot[b] : 0u;
    const uint32_t cv = b < bins ? (v + per - 1) / per : 0u;
    uint32_t all, call;
    const uint32_t ex = block_excl_scan<QT>(v, sh, &all);
    const uint32_t cex = block_excl_scan<QT>(cv, sh, &call);
    if (b < groups) {
      start[b] = carry + ex;
      chunk[b] = ccarry + cex;
      // the search blocks' map: block c works on the group b with
      // chunk[b] <= c < chunk[b + 1]
      for (uint32_t c = 0; c < cv; ++c) bmap[ccarry + cex + c] = static_cast<uint32_t>(b);
    }
    carry += all;
    ccarry += call;
  }
  if (threadIdx.x == 0) {
    start[groups] = carry;
    chunk[groups] = ccarry;
    A.w.oq_chunk[A.w.oq_bins + 1] = 0u;  // the staged search's work counter
  }
}

// The star pass: what star_start does, then each search to its group at an
// LDS-atomic slot (the order inside a group does not matter: each half lands
// where its search sits, and oq_pos says where); a lower turning point the
// LDS levels already finish is finished here, in a slot of the extra group.
// A table that fits the LDS whole (no level below the top) has no groups:
// its stars are searched here to the bottom and their records written in
// star order, the two slots of star i being 2i and 2i + 1.
template <class Ctx, typename MT, bool TO_STAGE, bool LF>
__global__ __launch_bounds__(QT) void k_oq_scatter(Ctx ctx, int corr) {
  extern __shared__ RPhi top[];
  __shared__ uint32_t cur[kTopEntries];
  __shared__ double shd[QT / 64];
  const ClusterArgs &A = ctx.args();
  const OrbitTop &tl = A.top;
  const RIndexCtl ictl = *A.w.rx_ctl;
  const int64_t n = ictl.n;
  const int64_t bins = query_bins(tl, n);
  const int64_t blk = ctx.block();
  const int64_t t = xcd_order(blk, ctx.nblocks());
  const int64_t k0 = t * kQueryTile;
  const Levels lv = levels_of(A.w);
  const RPhi *__restrict__ tab = lv.lev[0];
  const MS *__restrict__ ms = A.w.ms;
  OrbitRec *__restrict__ orec = A.w.orec;
  OrbitLo *__restrict__ res_lo = reinterpret_cast<OrbitLo *>(A.w.orec);
  OrbQuery *__restrict__ oq = A.w.oq;
  uint2 *__restrict__ pos = reinterpret_cast<uint2 *>(A.w.oq_pos);
  uint32_t fl = 0;
  if (k0 < n) {  // block-uniform
    if (bins == 0) {
      load_top(top, lv, tl, QT);
    } else {
      const uint32_t *__restrict__ row = A.w.oq_cnt + t * A.w.oq_bins;
      for (int b = threadIdx.x; b <= bins; b += QT) cur[b] = A.w.oq_start[b] + row[b];
    }
    __syncthreads();
    const int64_t k1 = k0 + kQueryTile < n ? k0 + kQueryTile : n;
    for (int j = 0; j < kQueryTile / QT && k0 + j * QT < n; ++j) {  // block-uniform
      const int64_t i = k0 + j * QT + threadIdx.x;
      double c_esc = 0.0, e_esc = 0.0;
      double E = 0.0, J = 0.0, J2 = 0.0;
      const bool bound =
          i < k1 &&
          star_start<MT, TO_STAGE, LF>(A, i, corr, E, J, J2, c_esc, e_esc, fl, bins == 0);
      if (i < k1 && !bound) pos[i] = make_uint2(kNoPos, kNoPos);  // it left
      if (bins == 0) {
        if (bound) {  // the whole table in LDS: the samples are the brackets
          const int32_t ii = static_cast<int32_t>(i);
          const int32_t kmin = top_descend(top, tl, lv.nlev, n, QNeg{2.0 * E, J2, ii});
          const int32_t kmax = top_descend(top, tl, lv.nlev, n, QNonNeg{2.0 * E, J2, ii});
          orec[i].lo = finalize_lo(tab, ms, kmin, E, J, J2);
          orec[i].hi = finalize_hi(tab, ms, n, kmax, E, J, J2);
          const uint32_t ui = static_cast<uint32_t>(i);
          pos[i] = make_uint2(2u * ui, 2u * ui + 1u);
        }
      } else if (bound) {
        const uint32_t code = A.w.oq_node[i];
        const int32_t t0 = static_cast<int32_t>(code & 0xFFFFu) - 1;
        const uint32_t t1 = code >> 16;
        const uint32_t ui = static_cast<uint32_t>(i);
        uint32_t plo;
        if (t0 < 0) {
          plo = atomicAdd(&cur[bins], 1u);
          res_lo[plo] = finalize_lo(tab, ms, -1, E, J, J2);
        } else {
          plo = atomicAdd(&cur[t0], 1u);
          oq[plo] = OrbQuery{E, J, ui, static_cast<uint32_t>(t0)};
        }
        const uint32_t phi_slot = atomicAdd(&cur[t1], 1u);
        oq[phi_slot] = OrbQuery{E, J, ui, t1 | kQueryHi};
        pos[i] = make_uint2(plo, phi_slot);
      }
      // escaper partials per 512 stars, as the direct form writes them
      esc_partials<QT>(c_esc, e_esc, shd, A.w.red_part, (k0 / QT) + j);
    }
  }
  or_status(A.s.sc, fl);
}

// The grouped searches.  Block b works on kQuerySearchChunk searches of one
// group (the first block of each group at oq_chunk): it stages the levels
// of the group's subtree that fit kSubEntries slots in LDS (padded as the
// top levels; one coalesced copy shared by all its searches), each lane
// descends them alone, the levels below go by groups of 8 lanes from global
// memory, and each lane finishes its own search.
template <class Ctx>
__global__ __launch_bounds__(QS) void k_oq_search(Ctx ctx) {
  __shared__ RPhi sub[kSubEntries];
  __shared__ GParams prm[QS];
  __shared__ int32_t soff[kMaxLevels];
  const ClusterArgs &A = ctx.args();
  const OrbitTop &tl = A.top;
  const RIndexCtl ictl = *A.w.rx_ctl;
  const int64_t n = ictl.n;
  const int64_t bins = query_bins(tl, n);
  if (bins == 0) return;
  const uint32_t *__restrict__ chunk = A.w.oq_chunk;
  const int64_t b = xcd_order(ctx.block(), ctx.nblocks());
  if (b >= static_cast<int64_t>(chunk[bins])) return;  // block-uniform
  const int64_t node = A.w.oq_bmap[b];  // the group of block b
  const int64_t q0 = A.w.oq_start[node] + (b - chunk[node]) * int64_t(kQuerySearchChunk);
  const int64_t qe = A.w.oq_start[node + 1];
  const int64_t q1 = q0 + kQuerySearchChunk < qe ? q0 + kQuerySearchChunk : qe;
  const Levels lv = levels_of(A.w);
  const int ltop = tl.ltop;
  // the subtree's levels ltop - 1 down to lsub, while they fit (padded)
  int lsub = ltop;
  {
    int64_t used = 0;
    while (lsub > 1) {
      const int64_t span = int64_t(1) << (3 * (ltop - lsub + 1));
      if (used + top_padded(span) > kSubEntries) break;
      used += top_padded(span);
      --lsub;
    }
  }
  if (threadIdx.x == 0) {
    int64_t used = 0;
    for (int L = ltop - 1; L >= lsub; --L) {
      soff[L] = static_cast<int32_t>(used);
      used += top_padded(int64_t(1) << (3 * (ltop - L)));
    }
  }
  __syncthreads();
  for (int L = ltop - 1; L >= lsub; --L) {
    const int64_t span = int64_t(1) << (3 * (ltop - L));
    const int64_t stride = int64_t(1) << (3 * L);
    const int64_t cnt = (n + stride - 1) >> (3 * L);
    const int64_t base = node * span;
    for (int64_t e = threadIdx.x; e < span; e += QS)
      if (base + e < cnt) sub[pad_slot(soff[L], e)] = lv.lev[L][base + e];
  }
  __syncthreads();
  GParams *wprm = prm + (threadIdx.x & ~63);
  const RPhi *__restrict__ tab = lv.lev[0];
  OrbitLo *__restrict__ res_lo = reinterpret_cast<OrbitLo *>(A.w.orec);
  OrbitHi *__restrict__ res_hi = reinterpret_cast<OrbitHi *>(A.w.orec);
  for (int64_t qb = q0; qb < q1; qb += QS) {  // block-uniform
    const int64_t qi = qb + threadIdx.x;
    const bool act = qi < q1;
    OrbQuery qr{0.0, 0.0, 0u, 0u};
    if (act) qr = A.w.oq[qi];
    const bool hi_b = (qr.node & kQueryHi) != 0u;
    const double J2 = qr.J * qr.J;
    const double twoE = 2.0 * qr.E;
    // the staged levels, per lane (the group's sample holds the predicate)
    const int32_t ci = static_cast<int32_t>(qr.i);
    const QAny pred{twoE, J2, hi_b ? -ci - 1 : ci};
    int32_t s = static_cast<int32_t>(node);
    if (act) {
      for (int L = ltop - 1; L >= lsub; --L) {
        const int32_t stride = int32_t(1) << (3 * L);
        const int32_t cnt = static_cast<int32_t>((n + stride - 1) >> (3 * L));
        const int32_t base = s * 8;
        const int32_t local = base - static_cast<int32_t>(node) * (int32_t(1) << (3 * (ltop - L)));
        s = base + node_last(sub + pad_slot(soff[L], local), cnt - base, base * stride, stride,
                             pred);
      }
    }
    const GParams mine{twoE, J2, hi_b ? -ci - 1 : ci, act ? s : -1};
    const int32_t k = group_descend1<GQAny>(lv, lsub - 1, n, mine, wprm);
    if (act) {  // the half where the search sits
      if (hi_b)
        res_hi[qi] = finalize_hi(tab, A.w.ms, n, k, qr.E, qr.J, J2);
      else
        res_lo[qi] = finalize_lo(tab, A.w.ms, k, qr.E, qr.J, J2);
    }
  }
}

// The grouped searches where a group's subtree spans at most kStagedLevels
// levels.  A work item is up to kStagedChunk searches of one group (the
// search blocks' map of k_oq_start).  Each resident block holds an item's
// whole subtree in LDS -- the levels below the top (padded as the top
// levels), level 0 itself and the (M, S) of its stars, each read once,
// coalesced -- and runs its searches, each lane alone from the group's
// sample down to its interval and on to the turning point: no table line
// is read per search.  A block takes its first item by its index and the
// next ones from a counter, and loads the next item's subtree into
// registers while the current item's searches run.
constexpr int SS = kStagedThreads;
constexpr int kStagedSub = (8 + 1 + 1) + (64 + 8 + 1) + (512 + 64 + 1);  // levels 3..1, padded
constexpr int kStagedL0 = kStagedSpan + kStagedSpan / 8 + 1;            // level 0, padded
constexpr int kStagedPer = kStagedSpan / SS;                            // level-0 entries a thread stages
static_assert(kStagedLevels == 4, "kStagedSub holds the padded levels 3..1");
static_assert(8 + 64 + 512 <= SS, "one subtree entry per thread");
static_assert(16 * (kStagedSub + kStagedL0 + kStagedSpan) + 64 <= 160 * 1024,
              "the staged subtree fits a workgroup's LDS");

// One item's subtree, held by the block's threads in registers on its way
// to LDS (as plain doubles, which the compiler keeps in registers).
struct StagedFetch {
  double sr, sphi;  // this thread's entry of the levels above level 0
  int32_t s_slot;   // its LDS slot (-1: none)
  double er[kStagedPer], ephi[kStagedPer], mM[kStagedPer], mS[kStagedPer];
  double r_next;    // thread 0: radius of the first star after the group (+inf: none)
};

__device__ __forceinline__ void staged_fetch(const ClusterArgs &A, const Levels &lv, int ltop,
                                             int64_t n, int64_t node, StagedFetch &f) {
  // thread x takes entry x of the levels ltop - 1 .. 1 laid end to end
  f.s_slot = -1;
  int64_t x = threadIdx.x, off = 0;
  for (int L = ltop - 1; L >= 1; --L) {
    const int64_t span = int64_t(1) << (3 * (ltop - L));
    const int64_t cnt = (n + (int64_t(1) << (3 * L)) - 1) >> (3 * L);
    if (x >= 0 && x < span && node * span + x < cnt) {
      const RPhi v = lv.lev[L][node * span + x];
      f.sr = v.r;
      f.sphi = v.phi;
      f.s_slot = static_cast<int32_t>(pad_slot(off, x));
    }
    x -= span;
    off += top_padded(span);
  }
  const int64_t span0 = int64_t(1) << (3 * ltop);
  const int64_t k0 = node * span0;
  const int64_t avail0 = n - k0 < span0 ? n - k0 : span0;
  const RPhi *__restrict__ tab = lv.lev[0];
  const MS *__restrict__ ms = A.w.ms;
#pragma unroll
  for (int u = 0; u < kStagedPer; ++u) {
    const int64_t e = threadIdx.x + u * SS;
    if (e < avail0) {
      const RPhi v = tab[k0 + e];
      const MS w = ms[k0 + e];
      f.er[u] = v.r;
      f.ephi[u] = v.phi;
      f.mM[u] = w.M;
      f.mS[u] = w.S;
    }
  }
  if (threadIdx.x == 0) f.r_next = k0 + span0 < n ? tab[k0 + span0].r : kInf;
}

template <class Ctx>
__global__ __launch_bounds__(SS) void k_oq_search_staged(Ctx ctx) {
  __shared__ RPhi sub[kStagedSub];
  __shared__ RPhi lv0[kStagedL0];
  __shared__ MS ms0[kStagedSpan];
  __shared__ double r_next;
  __shared__ int64_t claim;
  const ClusterArgs &A = ctx.args();
  const OrbitTop &tl = A.top;
  const int64_t n = A.w.rx_ctl->n;
  const int64_t bins = query_bins(tl, n);
  if (bins == 0) return;
  const uint32_t *__restrict__ chunk = A.w.oq_chunk;
  const uint32_t *__restrict__ qstart = A.w.oq_start;
  const uint32_t *__restrict__ bmap = A.w.oq_bmap;
  uint32_t *counter = A.w.oq_chunk + A.w.oq_bins + 1;
  const int64_t items = chunk[bins];
  const int64_t nb = ctx.nblocks();
  int64_t item = ctx.block();
  if (item >= items) return;  // block-uniform
  const Levels lv = levels_of(A.w);
  const int ltop = tl.ltop;  // 1 .. kStagedLevels
  const int64_t span0 = int64_t(1) << (3 * ltop);
  const int32_t n32 = static_cast<int32_t>(n);
  OrbitLo *__restrict__ res = reinterpret_cast<OrbitLo *>(A.w.orec);
  const OrbQuery *__restrict__ oq = A.w.oq;
  int64_t node = bmap[item];
  StagedFetch f;
  staged_fetch(A, lv, ltop, n, node, f);
  bool fresh = true;  // f holds the current item's subtree
  for (;;) {          // block-uniform
    const int64_t k0 = node * span0;
    if (fresh) {
      const int64_t avail0 = n - k0 < span0 ? n - k0 : span0;
      if (f.s_slot >= 0) sub[f.s_slot] = RPhi{f.sr, f.sphi};
#pragma unroll
      for (int u = 0; u < kStagedPer; ++u) {
        const int64_t e = threadIdx.x + u * SS;
        if (e < avail0) {
          lv0[pad_slot(0, e)] = RPhi{f.er[u], f.ephi[u]};
          ms0[e] = MS{f.mM[u], f.mS[u]};
        }
      }
      if (threadIdx.x == 0) r_next = f.r_next;
    }
    if (threadIdx.x == 0) claim = nb + static_cast<int64_t>(atomicAdd(counter, 1u));
    __syncthreads();
    // the next item: its subtree is read while this item's searches run
    const int64_t next = claim;
    const bool more = next < items;
    const int64_t next_node = more ? static_cast<int64_t>(bmap[next]) : -1;
    fresh = more && next_node != node;
    if (fresh) staged_fetch(A, lv, ltop, n, next_node, f);
    const int64_t q0 = qstart[node] + (item - chunk[node]) * int64_t(kStagedChunk);
    const int64_t qe = qstart[node + 1];
    const int64_t q1 = q0 + kStagedChunk < qe ? q0 + kStagedChunk : qe;
    // Lanes of a wavefront mix lower and upper searches, so the search runs
    // as one path for both: levels unrolled, every child read (inside the
    // staged arrays) and tested with selects, one root.
    int64_t qi = q0 + threadIdx.x;
    OrbQuery qr{0.0, 0.0, 0u, 0u};
    if (qi < q1) qr = oq[qi];
    for (int64_t qb = q0; qb < q1; qb += SS) {  // block-uniform
      const int64_t qn = qi + SS;
      OrbQuery nx{0.0, 0.0, 0u, 0u};
      if (qn < q1) nx = oq[qn];
      // a wavefront past the item's last search skips the round (the body
      // runs every lane unmasked, and the LDS is the bound)
      if (qb + static_cast<int64_t>(threadIdx.x & ~63u) >= q1) {
        qr = nx;
        qi = qn;
        continue;
      }
      const bool hi = (qr.node & kQueryHi) != 0u;
      const double J2 = qr.J * qr.J;
      const QSel pred{2.0 * qr.E, J2, static_cast<int32_t>(qr.i), hi};
      int32_t s = static_cast<int32_t>(node);
      int32_t off = 0;
#pragma unroll
      for (int L = kStagedLevels - 1; L >= 1; --L) {
        if (L < ltop) {  // uniform
          const int32_t stride = int32_t(1) << (3 * L);
          const int32_t cnt = static_cast<int32_t>((n + stride - 1) >> (3 * L));
          const int32_t span = int32_t(1) << (3 * (ltop - L));
          const int32_t base = s * 8;
          const int32_t local = base - static_cast<int32_t>(node) * span;
          s = base + node_last_sel(sub + pad_slot(off, local), cnt - base, base * stride, stride,
                                   pred);
          off += span + (span >> 3) + 1;
        }
      }
      // level 0: the interval itself, then its end radii and (M, S)
      const int32_t base = s * 8;
      const int32_t lb = base - static_cast<int32_t>(k0);
      const int32_t k = base + node_last_sel(lv0 + pad_slot(0, lb), n32 - base, base, 1, pred);
      const int32_t lk = k - static_cast<int32_t>(k0);
      const double rl = lv0[pad_slot(0, lk)].r;
      const double rh1 = lv0[pad_slot(0, lk + 1 < kStagedSpan ? lk + 1 : lk)].r;
      const double rh = k + 1 >= n32 ? kInf : (lk + 1 < span0 ? rh1 : r_next);
      const MS t = ms0[lk];
      double x = interval_root(hi, t, rl, rh, qr.E, J2);
      x = (!hi && J2 == 0.0) ? 0.0 : x;
      x = x < rl ? rl : (x > rh ? rh : x);
      // the 32-byte half: (E, rmin, dq, kmin) or (J, rmax, dq, kmax)
      OrbitLo o{};
      o.E = hi ? qr.J : qr.E;
      o.rmin = x;
      o.dq = (hi || J2 != 0.0) ? dq_of(t.M, k, x, J2) : 0.0;
      o.kmin = k;
      if (qi < q1) res[qi] = o;
      qr = nx;
      qi = qn;
    }
    if (!more) break;
    __syncthreads();  // every search done before the LDS takes the next subtree
    item = next;
    node = next_node;
  }
}

// Star i's orbit record: in star order (the direct form), or its two halves
// where the grouped form's searches left them.  False for a star that left.
__device__ __forceinline__ bool load_orbit(const ClusterArgs &A, int grouped, int64_t i,
                                           OrbitRec &o) {
  if (grouped) {
    const uint2 p = reinterpret_cast<const uint2 *>(A.w.oq_pos)[i];
    if (p.x == kNoPos) return false;
    o.lo = reinterpret_cast<const OrbitLo *>(A.w.orec)[p.x];
    o.hi = reinterpret_cast<const OrbitHi *>(A.w.orec)[p.y];
  } else {
    o = A.w.orec[i];
  }
  return o.lo.E < 0.0;  // the direct form marks a star that left by E >= 0 (or NaN)
}

// Waves per SIMD: the FP64 form needs ~120 VGPRs and runs spill-free at 4
// (1.18 ms at N = 1e7, against 1.32 ms at 5 with 56-80 bytes of spill per
// lane); the mixed form fits 96 at 5 (a 12-byte spill, and 1.15 against
// 1.17 ms at 4).
template <class Ctx, typename MT, bool TO_STAGE, bool MIXED, bool LF>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(MIXED ? 5 : 4)))
void k_orbit_trials(Ctx ctx, uint32_t step_arg, int32_t trial_cap, int corr,
                    double bound_factor, int grouped) {
  __shared__ double shd[NT / 64];
  // stars of each wavefront's chunk finished without trials (kept apart so
  // that their code does not hold registers in the trial loop)
  __shared__ uint32_t deferred[NT / 64][kMaxTrialChunk];
  __shared__ uint32_t n_deferred[NT / 64];
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
  const int64_t chunk = A.w.trial_chunk;  // stars per wavefront
  const int64_t c_end0 = (wave + 1) * chunk;
  const int64_t c_end = c_end0 < n ? c_end0 : n;
  int64_t cursor = wave * chunk;  // wave-uniform
  uint32_t c_tr = 0, c_viol = 0, c_cap = 0;
  uint32_t fl = 0;

  const int wv = threadIdx.x >> 6;
  if (lane == 0) n_deferred[wv] = 0u;
  __builtin_amdgcn_wave_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);

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
        OrbitRec o;
        if (load_orbit(A, grouped, mine, o)) {  // else an escaper, already sent out
          // the rejection bound: F = bound_factor * the larger endpoint
          // value of g(s), 2 r_a / |dQ/dr| under the square root
          const double oJ = o.hi.J, oJ2 = oJ * oJ;
          const double orc = 0.5 * (o.hi.rmax + o.lo.rmin);
          const double ora = 0.5 * (o.hi.rmax - o.lo.rmin);
          double oF = -1.0;
          if (ora > 0.0) {
            const double glo = (oJ2 != 0.0) ? sqrt(2.0 * ora / fabs(o.lo.dq)) : 0.0;
            const double ghi = sqrt(2.0 * ora / fabs(o.hi.dq));
            oF = bound_factor * (glo > ghi ? glo : ghi);
            if (!(oF > 0.0 && oF < kInf)) {
              oF = -1.0;
              fl |= CMC_ST_NUMERIC;  // finished at the orbit's centre, below
            }
          }
          if (oF > 0.0) {
            busy = true;
            i = mine;
            E = o.lo.E;
            J = oJ;
            J2 = oJ2;
            rc = orc;
            ra = ora;
            F = oF;
            kmin = o.lo.kmin;
            kmax = o.hi.kmax;
            sid = id[mine];
            j = 0;
            if (LF) lg = load_lfsr(A.s.rng, mine);
          } else {
            // a point orbit (or no usable bound): finished without trials
            // after the loop
            const uint32_t slot = atomicAdd(&n_deferred[wv], 1u);
            deferred[wv][slot] = static_cast<uint32_t>(mine - wave * chunk);
          }
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
  // the deferred stars: the new radius is rdone (r_min, or the orbit's
  // centre when the bound is unusable), with no trial
  __builtin_amdgcn_wave_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  const uint32_t nd = n_deferred[wv];
  for (uint32_t d = lane; d < nd; d += 64) {
    const int64_t mine = wave * chunk + deferred[wv][d];
    OrbitRec o;
    load_orbit(A, grouped, mine, o);
    const double oJ = o.hi.J, oJ2 = oJ * oJ;
    const double ora = 0.5 * (o.hi.rmax - o.lo.rmin);
    const double rdone = ora > 0.0 ? 0.5 * (o.hi.rmax + o.lo.rmin) : o.lo.rmin;
    const double rn = rdone + 0.0;
    const int64_t kn = interval_in(ix, ictl, rn, o.lo.kmin, o.hi.kmax);
    const double phn = phi_in(lv, ms, kn, rn);
    const double qn = 2.0 * o.lo.E - 2.0 * phn - (oJ2 == 0.0 ? 0.0 : oJ2 / (rn * rn));
    if (corr) pn[mine] = phn;
    U4 ws;
    if (LF) {
      Lfsr g = load_lfsr(A.s.rng, mine);
      ws = lfsr_block(g);
      put_lfsr<TO_STAGE>(A, mine, g);
    } else {
      ws = philox(id[mine], step, kSign, 0u, seed);
    }
    double vrn, vtn;
    finish(rn, qn, oJ, oJ2, ws.x, vrn, vtn, fl);
    emit<TO_STAGE>(mine, rn, vrn, vtn, m[mine], id[mine], rindex_last_le(ix, ictl, rn) + 1,
                   r_new, vr, vt, stage, keys, bkey);
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

// One block per cluster: the cluster's escaper and trial partials.
template <class Ctx>
__global__ __launch_bounds__(FT) void k_orbit_sum(Ctx ctx) {
  __shared__ double sh[FT / 64];
  const ClusterArgs &A = ctx.args();
  const double *__restrict__ pa = A.w.red_part;
  const double *__restrict__ pb = A.w.red_part + 2 * A.w.star_blocks;
  const int64_t na = cdiv(A.w.rx_ctl->n, 512);  // escaper partials, per 512 stars
  const int64_t nb = blocks_of(kShTrials, A.w, A.s.cap);
  cmc_scalars *__restrict__ sc = A.s.sc;
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
  for (int64_t b = threadIdx.x; b < na; b += FT) {
    v[0] += pa[2 * b];
    v[4] += pa[2 * b + 1];
  }
#pragma unroll 8
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
hipError_t run2(const L &l, const cmc_params &p, int corr, bool sorted, hipStream_t st) {
  const int32_t cap = p.trial_cap > 0 ? p.trial_cap : 10000;
  const double bf = p.bound_factor > 0.0 ? p.bound_factor : 1.2;
  using Ct = decltype(l.ctx(kShTrials));
  const size_t top_bytes = sizeof(RPhi) * l.top_entries();
  k_phi_bounds<<<l.grid(kShDiag), NT, 0, st>>>(l.ctx(kShDiag));
  if (sorted) {
    using Cq = decltype(l.ctx(kShQTile));
    k_oq_hist<<<l.grid(kShQTile), QT, top_bytes, st>>>(l.ctx(kShQTile));
    k_oq_colscan<<<l.grid(kShQGroup), CT, 0, st>>>(l.ctx(kShQGroup));
    k_oq_start<<<l.grid(kShOne), QT, 0, st>>>(l.ctx(kShOne));
    k_oq_scatter<Cq, MT, TO_STAGE, LF>
        <<<l.grid(kShQTile), QT, l.flat_top() ? top_bytes : 0, st>>>(l.ctx(kShQTile), corr);
    // by the subtree's depth (an ensemble may hold both kinds)
    if (l.grid(kShQSearch) > 0)
      k_oq_search<<<l.grid(kShQSearch), QS, 0, st>>>(l.ctx(kShQSearch));
    if (l.grid(kShQStaged) > 0)
      k_oq_search_staged<<<l.grid(kShQStaged), SS, 0, st>>>(l.ctx(kShQStaged));
  } else {
    using Cb = decltype(l.ctx(kShBracket));
    k_orbit_bracket<Cb, MT, TO_STAGE, LF><<<l.grid(kShBracket), BT, top_bytes, st>>>(
        l.ctx(kShBracket), corr);
  }
  const int grouped = sorted ? 1 : 0;
  if (p.precision == CMC_MIXED)
    k_orbit_trials<Ct, MT, TO_STAGE, true, LF><<<l.grid(kShTrials), NT, 0, st>>>(
        l.ctx(kShTrials), p.step, cap, corr, bf, grouped);
  else
    k_orbit_trials<Ct, MT, TO_STAGE, false, LF><<<l.grid(kShTrials), NT, 0, st>>>(
        l.ctx(kShTrials), p.step, cap, corr, bf, grouped);
  k_orbit_sum<<<l.grid(kShOne), FT, 0, st>>>(l.ctx(kShOne));
  return hipGetLastError();
}

}  // namespace

static_assert(sizeof(OrbitRec) == 64 && sizeof(OrbitLo) == 32 && sizeof(OrbitHi) == 32,
              "orbit record layout");
static_assert(sizeof(OrbQuery) == 24, "search record layout");
static_assert(BT == kBracketThreads && QT == BT, "launch shapes: escaper partials per 512 stars");

OrbitTop orbit_top(const Workspace &w, int64_t cap) { return top_levels(w.nlev, cap); }

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
  const bool sorted = sorted_searches(t);
  return dispatch(t, [&](const auto &l) {
    using L = std::decay_t<decltype(l)>;
    if (lf) {
      if (m_f32)
        return to_stage ? run2<L, float, true, true>(l, p, c, sorted, st)
                        : run2<L, float, false, true>(l, p, c, sorted, st);
      return to_stage ? run2<L, double, true, true>(l, p, c, sorted, st)
                      : run2<L, double, false, true>(l, p, c, sorted, st);
    }
    if (m_f32)
      return to_stage ? run2<L, float, true, false>(l, p, c, sorted, st)
                      : run2<L, float, false, false>(l, p, c, sorted, st);
    return to_stage ? run2<L, double, true, false>(l, p, c, sorted, st)
                    : run2<L, double, false, false>(l, p, c, sorted, st);
  });
}

}  // namespace cmc

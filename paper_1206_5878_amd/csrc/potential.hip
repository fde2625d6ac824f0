// potential.hip -- the cumulative-mass potential (arXiv:1206.5878, Sec. 2.1
// step 1): for sorted radii, Phi_k = -(M_k / r_k + S_k) with M_k the
// inclusive prefix of m and S_k the exclusive suffix of m/r.  Device-wide
// scan in three deterministic passes: per-tile sums, a one-block scan of the
// tile sums (forward for M, backward for S), and a per-tile apply that adds
// the carries to in-tile scans.  A tile is 4 rounds of 256 consecutive stars,
// thread t holding star t of each round, so every load and store of a wave
// is one contiguous run; the in-tile scans are block scans per round.
//
// Sums: FP64 in the FP64 form.  The mixed form forms m / r in FP32 and sums
// inside a tile in FP32 with a compensation term (each partial sum an
// unevaluated pair hi + lo, two-sum on every addition, about 48 significant
// bits); the tile sums and the carries across tiles are FP64.
// HBM-bound: reads r and m, writes the orbit table ((r, Phi) and (M, S) per
// star plus the sampled search levels) and, for the standalone call, the
// state's phi, mcum, ssuf.
#include <type_traits>

#include "cmc_internal.hpp"

namespace cmc {
namespace {

constexpr int PT = kBlock;
constexpr int PJ = kPotTile / PT;  // rounds of PT consecutive stars per tile

// ---------------------------------------------------------------- accumulators
// FP64 sums.
struct D1 {
  double v;
};
__device__ __forceinline__ D1 acc_add(D1 a, D1 b) { return D1{a.v + b.v}; }
__device__ __forceinline__ D1 acc_of(double x) { return D1{x}; }
__device__ __forceinline__ double acc_val(D1 a) { return a.v; }
__device__ __forceinline__ D1 acc_shfl_up(D1 a, int o) { return D1{__shfl_up(a.v, o, 64)}; }
__device__ __forceinline__ D1 acc_shfl_down(D1 a, int o) { return D1{__shfl_down(a.v, o, 64)}; }

// Compensated FP32 sums: hi + lo, renormalised after every addition
// (Knuth's two-sum on the leading parts, the trailing parts added).
struct F2 {
  float hi, lo;
};
__device__ __forceinline__ F2 acc_add(F2 a, F2 b) {
  const float s = a.hi + b.hi;
  const float bb = s - a.hi;
  const float err = (a.hi - (s - bb)) + (b.hi - bb);
  const float t = err + (a.lo + b.lo);
  const float h = s + t;
  return F2{h, t - (h - s)};
}
__device__ __forceinline__ F2 acc_of(float x) { return F2{x, 0.0f}; }
__device__ __forceinline__ double acc_val(F2 a) {
  return static_cast<double>(a.hi) + static_cast<double>(a.lo);
}
__device__ __forceinline__ F2 acc_shfl_up(F2 a, int o) {
  return F2{__shfl_up(a.hi, o, 64), __shfl_up(a.lo, o, 64)};
}
__device__ __forceinline__ F2 acc_shfl_down(F2 a, int o) {
  return F2{__shfl_down(a.hi, o, 64), __shfl_down(a.lo, o, 64)};
}

// The form's accumulator and the value type of m / r.
template <bool MIXED>
using Acc = std::conditional_t<MIXED, F2, D1>;
template <bool MIXED>
using Val = std::conditional_t<MIXED, float, double>;

template <bool MIXED>
__device__ __forceinline__ Val<MIXED> m_over_r(double m, double r) {
  if constexpr (MIXED)
    return static_cast<float>(m) / static_cast<float>(r);
  else
    return m / r;
}

// Over the block, in thread order: the exclusive prefix of a and the
// exclusive suffix of b, with both block totals, through one LDS exchange.
template <int NTB, class A>
__device__ __forceinline__ void block_scan_pair(A a, A b, A *sh, A &pa, A &sb, A &ta, A &tb) {
  constexpr int NW = NTB / 64;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  A ia = a, ib = b;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const A ua = acc_shfl_up(ia, o);
    const A ub = acc_shfl_down(ib, o);
    if (l >= o) ia = acc_add(ua, ia);
    if (l + o < 64) ib = acc_add(ib, ub);
  }
  A ea = acc_shfl_up(ia, 1);
  A eb = acc_shfl_down(ib, 1);
  const A zero = acc_of(Val<std::is_same_v<A, F2>>(0));
  if (l == 0) ea = zero;
  if (l == 63) eb = zero;
  if (l == 63) sh[w] = ia;
  if (l == 0) sh[NW + w] = ib;
  __syncthreads();
  A ba = zero, bb = zero, sa = zero;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    const A x = sh[i];
    if (i < w) ba = acc_add(ba, x);
    sa = acc_add(sa, x);
  }
  A sbt = zero;
#pragma unroll
  for (int i = NW - 1; i >= 0; --i) {
    const A y = sh[NW + i];
    if (i > w) bb = acc_add(bb, y);
    sbt = acc_add(sbt, y);
  }
  __syncthreads();
  pa = acc_add(ba, ea);
  sb = acc_add(bb, eb);
  ta = sa;
  tb = sbt;
}

template <class Ctx, typename MT, bool MIXED>
__global__ __launch_bounds__(PT) void k_pot_tile_sums(Ctx ctx) {
  using A = Acc<MIXED>;
  __shared__ A sh[2 * (PT / 64)];
  const ClusterArgs &A_ = ctx.args();
  const double *__restrict__ r = A_.s.r;
  const MT *__restrict__ m = static_cast<const MT *>(A_.s.m);
  const int64_t n = A_.s.sc->n;
  const int64_t tiles = A_.w.pot_tiles;
  const int64_t t = ctx.block();
  const int64_t base = t * kPotTile + threadIdx.x;
  A sm = acc_of(Val<MIXED>(0)), sq = sm;
#pragma unroll
  for (int j = 0; j < PJ; ++j) {
    const int64_t k = base + j * PT;
    if (k < n) {
      const double mk = load_mass(m, k);
      sm = acc_add(sm, acc_of(static_cast<Val<MIXED>>(mk)));
      sq = acc_add(sq, acc_of(m_over_r<MIXED>(mk, r[k])));
    }
  }
  A pa, sb, tm, tq;
  block_scan_pair<PT>(sm, sq, sh, pa, sb, tm, tq);
  if (threadIdx.x == 0) {
    A_.w.pot_tsum[t] = acc_val(tm);
    A_.w.pot_tsum[tiles + t] = acc_val(tq);
  }
}

constexpr int ST = 1024;
constexpr int SQ = 16;  // tile sums a thread of the tile scan holds in registers

// One block per cluster; thread t scans tiles [t per, (t+1) per).  Up to SQ
// tiles per thread are loaded at once (N up to SQ * ST * kPotTile stars);
// beyond that the thread walks its range.
template <class Ctx>
__global__ __launch_bounds__(ST) void k_pot_tile_scan(Ctx ctx) {
  __shared__ double sh[ST / 64];
  const ClusterArgs &A = ctx.args();
  const double *__restrict__ tsum = A.w.pot_tsum;
  double *__restrict__ carry = A.w.pot_carry;
  const int64_t tiles = A.w.pot_tiles;
  const int64_t per = (tiles + ST - 1) / ST;
  const int64_t b = static_cast<int64_t>(threadIdx.x) * per;
  const int64_t e = b + per < tiles ? b + per : tiles;
  if (per <= SQ) {
    double vm[SQ], vq[SQ];
    double sm = 0.0, sq = 0.0;
#pragma unroll
    for (int q = 0; q < SQ; ++q) {
      const bool ok = b + q < e;
      vm[q] = ok ? tsum[b + q] : 0.0;
      vq[q] = ok ? tsum[tiles + b + q] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < SQ; ++q) {
      sm += vm[q];
      sq += vq[q];
    }
    double acc = block_excl_scan<ST>(sm, sh, static_cast<double *>(nullptr));
#pragma unroll
    for (int q = 0; q < SQ; ++q) {
      if (b + q < e) carry[b + q] = acc;
      acc += vm[q];
    }
    acc = block_excl_suffix<ST>(sq, sh, static_cast<double *>(nullptr));
#pragma unroll
    for (int q = SQ - 1; q >= 0; --q) {
      if (b + q < e) {
        carry[tiles + b + q] = acc;
        acc += vq[q];
      }
    }
    return;
  }
  double sm = 0.0, sq = 0.0;
  for (int64_t k = b; k < e; ++k) {
    sm += tsum[k];
    sq += tsum[tiles + k];
  }
  const double pm = block_excl_scan<ST>(sm, sh, static_cast<double *>(nullptr));
  const double pq = block_excl_suffix<ST>(sq, sh, static_cast<double *>(nullptr));
  double acc = pm;
  for (int64_t k = b; k < e; ++k) {
    carry[k] = acc;
    acc += tsum[k];
  }
  acc = pq;
  for (int64_t k = e - 1; k >= b; --k) {
    carry[tiles + k] = acc;
    acc += tsum[tiles + k];
  }
}

// PUBLIC: write the state's phi, mcum, ssuf; TABLE: write the orbit table in
// the workspace.
template <class Ctx, typename MT, bool PUBLIC, bool MIXED, bool TABLE = true>
__global__ __launch_bounds__(PT) void k_pot_apply(Ctx ctx) {
  using A = Acc<MIXED>;
  __shared__ A sh[2 * (PT / 64)];
  const ClusterArgs &A_ = ctx.args();
  const double *__restrict__ r = A_.s.r;
  const MT *__restrict__ m = static_cast<const MT *>(A_.s.m);
  const double *__restrict__ carry = A_.w.pot_carry;
  const int64_t n = A_.s.sc->n;
  const int64_t tiles = A_.w.pot_tiles;
  const Levels lv = levels_of(A_.w);
  const int64_t t = ctx.block();
  const int64_t base = t * kPotTile + threadIdx.x;
  double rr[PJ], mk[PJ];
#pragma unroll
  for (int j = 0; j < PJ; ++j) {
    const int64_t k = base + j * PT;
    const bool ok = k < n;
    rr[j] = ok ? r[k] : 1.0;
    mk[j] = ok ? load_mass(m, k) : 0.0;
  }
  // M: inclusive prefix, round by round; S: exclusive suffix inside each
  // round, then the later rounds' totals (the later tiles' carry is added
  // in FP64 below)
  A pm[PJ], sq[PJ], tq[PJ];
  A cm = acc_of(Val<MIXED>(0));
#pragma unroll
  for (int j = 0; j < PJ; ++j) {
    const A mj = acc_of(static_cast<Val<MIXED>>(mk[j]));
    A ex, tm;
    block_scan_pair<PT>(mj, acc_of(m_over_r<MIXED>(mk[j], rr[j])), sh, ex, sq[j], tm, tq[j]);
    pm[j] = acc_add(cm, acc_add(ex, mj));
    cm = acc_add(cm, tm);
  }
  A cs = acc_of(Val<MIXED>(0));
#pragma unroll
  for (int j = PJ - 1; j >= 0; --j) {
    sq[j] = acc_add(sq[j], cs);
    cs = acc_add(cs, tq[j]);
  }
  const double cmt = carry[t], cqt = carry[tiles + t];
#pragma unroll
  for (int j = 0; j < PJ; ++j) {
    const int64_t k = base + j * PT;
    if (k < n) {
      const double M = cmt + acc_val(pm[j]);
      const double S = cqt + acc_val(sq[j]);
      const double ph = -(M / rr[j] + S);
      if (PUBLIC) {
        A_.s.mcum[k] = M;
        A_.s.ssuf[k] = S;
        A_.s.phi[k] = ph;
      }
      if (TABLE) put_table(lv, A_.w.ms, k, rr[j], ph, M, S);
    }
  }
}

template <class L, typename MT, bool MIXED>
hipError_t run(const L &l, bool pub, hipStream_t st) {
  k_pot_tile_sums<decltype(l.ctx(kShPotTile)), MT, MIXED>
      <<<l.grid(kShPotTile), PT, 0, st>>>(l.ctx(kShPotTile));
  k_pot_tile_scan<<<l.grid(kShOne), ST, 0, st>>>(l.ctx(kShOne));
  if (pub)
    k_pot_apply<decltype(l.ctx(kShPotTile)), MT, true, MIXED>
        <<<l.grid(kShPotTile), PT, 0, st>>>(l.ctx(kShPotTile));
  else
    k_pot_apply<decltype(l.ctx(kShPotTile)), MT, false, MIXED>
        <<<l.grid(kShPotTile), PT, 0, st>>>(l.ctx(kShPotTile));
  return hipGetLastError();
}

// The state's phi, mcum, ssuf only, with no orbit table (a workspace holding
// just the scan's tile sums and carries).
template <class L, typename MT, bool MIXED>
hipError_t run_public_only(const L &l, hipStream_t st) {
  k_pot_tile_sums<decltype(l.ctx(kShPotTile)), MT, MIXED>
      <<<l.grid(kShPotTile), PT, 0, st>>>(l.ctx(kShPotTile));
  k_pot_tile_scan<<<l.grid(kShOne), ST, 0, st>>>(l.ctx(kShOne));
  k_pot_apply<decltype(l.ctx(kShPotTile)), MT, true, MIXED, false>
      <<<l.grid(kShPotTile), PT, 0, st>>>(l.ctx(kShPotTile));
  return hipGetLastError();
}

}  // namespace

hipError_t launch_potential_public_only(const Target &t, bool m_f32, int precision,
                                        hipStream_t st) {
  return dispatch(t, [&](const auto &l) {
    using L = std::decay_t<decltype(l)>;
    const bool mx = precision == CMC_MIXED;
    if (m_f32)
      return mx ? run_public_only<L, float, true>(l, st) : run_public_only<L, float, false>(l, st);
    return mx ? run_public_only<L, double, true>(l, st) : run_public_only<L, double, false>(l, st);
  });
}

hipError_t launch_potential(const Target &t, bool m_f32, int precision, bool public_arrays,
                            hipStream_t st) {
  return dispatch(t, [&](const auto &l) {
    const bool mx = precision == CMC_MIXED;
    if (m_f32)
      return mx ? run<std::decay_t<decltype(l)>, float, true>(l, public_arrays, st)
                : run<std::decay_t<decltype(l)>, float, false>(l, public_arrays, st);
    return mx ? run<std::decay_t<decltype(l)>, double, true>(l, public_arrays, st)
              : run<std::decay_t<decltype(l)>, double, false>(l, public_arrays, st);
  });
}

}  // namespace cmc

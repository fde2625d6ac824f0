// potential.hip -- the cumulative-mass potential (arXiv:1206.5878, Sec. 2.1
// step 1): for sorted radii, Phi_k = -(M_k / r_k + S_k) with M_k the
// inclusive prefix of m and S_k the exclusive suffix of m/r.  Device-wide
// scan in three deterministic passes: per-tile sums, a one-block scan of the
// tile sums (forward for M, backward for S), and a per-tile apply that adds
// the carries to in-tile scans.  A tile is 4 rounds of 256 consecutive stars,
// thread t holding star t of each round, so every load and store of a wave
// is one contiguous run; the in-tile scans are block scans per round.  The
// mixed form forms m / r in FP32; every sum is FP64.  HBM-bound: reads r and
// m, writes the orbit table ((r, Phi) and (M, S) per star plus the sampled
// search levels) and, for the standalone call, the state's phi, mcum, ssuf.
#include <type_traits>

#include "cmc_internal.hpp"

namespace cmc {
namespace {

constexpr int PT = kBlock;
constexpr int PJ = kPotTile / PT;  // rounds of PT consecutive stars per tile

// m / r: FP64, or FP32 for the mixed form.
template <bool MIXED>
__device__ __forceinline__ double m_over_r(double m, double r) {
  return MIXED ? static_cast<double>(static_cast<float>(m) / static_cast<float>(r)) : m / r;
}

// Over the block, in thread order: the exclusive prefix of a and the exclusive
// suffix of b, with both block totals, through one LDS exchange.  The sums
// run in the same order as block_excl_scan and block_excl_suffix.
__device__ __forceinline__ void block_scan_pair(double a, double b, double *sh, double &pa,
                                                double &sb, double &ta, double &tb) {
  constexpr int NW = PT / 64;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double ia = wave_incl_scan(a);
  const double ib = wave_incl_suffix(b);
  double ea = __shfl_up(ia, 1, 64);
  double eb = __shfl_down(ib, 1, 64);
  if (l == 0) ea = 0.0;
  if (l == 63) eb = 0.0;
  if (l == 63) sh[w] = ia;
  if (l == 0) sh[NW + w] = ib;
  __syncthreads();
  double ba = 0.0, bb = 0.0, sa = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    const double x = sh[i];
    if (i < w) ba += x;
    sa += x;
  }
  double sbt = 0.0;
#pragma unroll
  for (int i = NW - 1; i >= 0; --i) {
    const double y = sh[NW + i];
    if (i > w) bb += y;
    sbt += y;
  }
  __syncthreads();
  pa = ba + ea;
  sb = bb + eb;
  ta = sa;
  tb = sbt;
}

template <class Ctx, typename MT, bool MIXED>
__global__ __launch_bounds__(PT) void k_pot_tile_sums(Ctx ctx) {
  __shared__ double sh[PT / 64];
  const ClusterArgs &A = ctx.args();
  const double *__restrict__ r = A.s.r;
  const MT *__restrict__ m = static_cast<const MT *>(A.s.m);
  const int64_t n = A.s.sc->n;
  const int64_t tiles = A.w.pot_tiles;
  const int64_t t = ctx.block();
  const int64_t base = t * kPotTile + threadIdx.x;
  double sm = 0.0, sq = 0.0;
#pragma unroll
  for (int j = 0; j < PJ; ++j) {
    const int64_t k = base + j * PT;
    if (k < n) {
      const double mk = load_mass(m, k);
      sm += mk;
      sq += m_over_r<MIXED>(mk, r[k]);
    }
  }
  const double tm = block_sum<PT>(sm, sh);
  const double tq = block_sum<PT>(sq, sh);
  if (threadIdx.x == 0) {
    A.w.pot_tsum[t] = tm;
    A.w.pot_tsum[tiles + t] = tq;
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
  __shared__ double sh[2 * (PT / 64)];
  const ClusterArgs &A = ctx.args();
  const double *__restrict__ r = A.s.r;
  const MT *__restrict__ m = static_cast<const MT *>(A.s.m);
  const double *__restrict__ carry = A.w.pot_carry;
  const int64_t n = A.s.sc->n;
  const int64_t tiles = A.w.pot_tiles;
  const Levels lv = levels_of(A.w);
  const int64_t t = ctx.block();
  const int64_t base = t * kPotTile + threadIdx.x;
  double rr[PJ], mk[PJ], q[PJ];
#pragma unroll
  for (int j = 0; j < PJ; ++j) {
    const int64_t k = base + j * PT;
    const bool ok = k < n;
    rr[j] = ok ? r[k] : 1.0;
    mk[j] = ok ? load_mass(m, k) : 0.0;
    q[j] = m_over_r<MIXED>(mk[j], rr[j]);
  }
  // M: inclusive prefix, round by round; S: exclusive suffix inside each
  // round, then the later rounds' totals and the later tiles' carry
  double M[PJ], S[PJ], tq[PJ];
  double cm = carry[t];
#pragma unroll
  for (int j = 0; j < PJ; ++j) {
    double ex, tm;
    block_scan_pair(mk[j], q[j], sh, ex, S[j], tm, tq[j]);
    M[j] = cm + (ex + mk[j]);
    cm += tm;
  }
  double cq = carry[tiles + t];
#pragma unroll
  for (int j = PJ - 1; j >= 0; --j) {
    S[j] += cq;
    cq += tq[j];
  }
#pragma unroll
  for (int j = 0; j < PJ; ++j) {
    const int64_t k = base + j * PT;
    if (k < n) {
      const double ph = -(M[j] / rr[j] + S[j]);
      if (PUBLIC) {
        A.s.mcum[k] = M[j];
        A.s.ssuf[k] = S[j];
        A.s.phi[k] = ph;
      }
      if (TABLE) put_table(lv, A.w.ms, k, rr[j], ph, M[j], S[j]);
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

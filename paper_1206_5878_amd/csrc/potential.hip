// potential.hip -- the cumulative-mass potential (arXiv:1206.5878, Sec. 2.1
// step 1): for sorted radii, Phi_k = -(M_k / r_k + S_k) with M_k the
// inclusive prefix of m and S_k the exclusive suffix of m/r.  Device-wide
// scan in three deterministic passes: per-tile sums, a one-block scan of the
// tile sums (forward for M, backward for S), and a per-tile apply that adds
// the carries to in-tile scans.  The mixed form sums each thread's run of 8
// stars in compensated FP32 and keeps the block scans and carries in FP64.
// HBM-bound: reads r and m, writes the
// orbit table ((r, Phi) and (M, S) per star plus the sampled search levels)
// and, for the standalone call, the state's phi, mcum, ssuf.
#include <type_traits>

#include "cmc_internal.hpp"

namespace cmc {
namespace {

constexpr int PT = kBlock;
constexpr int PJ = kPotTile / kBlock;  // 8 consecutive stars per thread

// Error-free float addition (Knuth's two-sum): s + e == a + b exactly.
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Running sum of a thread's run: FP64, or compensated FP32 (sum + error term,
// read out in FP64) for the mixed form.
template <bool MIXED>
struct Acc {
  double d = 0.0;
  float s = 0.0f, e = 0.0f;
  __device__ __forceinline__ void add(double x) {
    if (MIXED) {
      float t, err;
      two_sum(s, static_cast<float>(x), t, err);
      s = t;
      e += err;
    } else {
      d += x;
    }
  }
  __device__ __forceinline__ double value() const {
    return MIXED ? static_cast<double>(s) + static_cast<double>(e) : d;
  }
};

// m / r: FP64, or FP32 for the mixed form.
template <bool MIXED>
__device__ __forceinline__ double m_over_r(double m, double r) {
  return MIXED ? static_cast<double>(static_cast<float>(m) / static_cast<float>(r)) : m / r;
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
  const int64_t base = t * kPotTile + static_cast<int64_t>(threadIdx.x) * PJ;
  Acc<MIXED> sm, sq;
#pragma unroll
  for (int j = 0; j < PJ; ++j) {
    const int64_t k = base + j;
    if (k < n) {
      const double mk = load_mass(m, k);
      sm.add(mk);
      sq.add(m_over_r<MIXED>(mk, r[k]));
    }
  }
  const double tm = block_sum<PT>(sm.value(), sh);
  const double tq = block_sum<PT>(sq.value(), sh);
  if (threadIdx.x == 0) {
    A.w.pot_tsum[t] = tm;
    A.w.pot_tsum[tiles + t] = tq;
  }
}

constexpr int ST = 1024;

// One block per cluster.
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

template <class Ctx, typename MT, bool PUBLIC, bool MIXED>
__global__ __launch_bounds__(PT) void k_pot_apply(Ctx ctx) {
  __shared__ double sh[PT / 64];
  const ClusterArgs &A = ctx.args();
  const double *__restrict__ r = A.s.r;
  const MT *__restrict__ m = static_cast<const MT *>(A.s.m);
  const double *__restrict__ carry = A.w.pot_carry;
  const int64_t n = A.s.sc->n;
  const int64_t tiles = A.w.pot_tiles;
  const Levels lv = levels_of(A.w);
  const int64_t t = ctx.block();
  const int64_t base = t * kPotTile + static_cast<int64_t>(threadIdx.x) * PJ;
  double rr[PJ], pm[PJ], sq[PJ];
  Acc<MIXED> am;
#pragma unroll
  for (int j = 0; j < PJ; ++j) {
    const int64_t k = base + j;
    const bool ok = k < n;
    rr[j] = ok ? r[k] : 1.0;
    const double mk = ok ? load_mass(m, k) : 0.0;
    am.add(mk);
    pm[j] = am.value();  // inclusive prefix inside the thread
    sq[j] = m_over_r<MIXED>(mk, rr[j]);
  }
  const double tm = am.value();
  Acc<MIXED> aq;
#pragma unroll
  for (int j = PJ - 1; j >= 0; --j) {  // exclusive suffix inside the thread
    const double q = sq[j];
    sq[j] = aq.value();
    aq.add(q);
  }
  const double tq = aq.value();
  const double em = block_excl_scan<PT>(tm, sh, static_cast<double *>(nullptr));
  const double eq = block_excl_suffix<PT>(tq, sh, static_cast<double *>(nullptr));
  const double cm = carry[t] + em;
  const double cq = carry[tiles + t] + eq;
#pragma unroll
  for (int j = 0; j < PJ; ++j) {
    const int64_t k = base + j;
    if (k < n) {
      const double M = cm + pm[j];
      const double S = cq + sq[j];
      const double ph = -(M / rr[j] + S);
      if (PUBLIC) {
        A.s.mcum[k] = M;
        A.s.ssuf[k] = S;
        A.s.phi[k] = ph;
      }
      put_table(lv, A.w.ms, k, rr[j], ph, M, S);
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

}  // namespace

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

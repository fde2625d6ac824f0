// potential.hip -- the cumulative-mass potential (arXiv:1206.5878, Sec. 2.1
// step 1): for sorted radii, Phi_k = -(M_k / r_k + S_k) with M_k the
// inclusive prefix of m and S_k the exclusive suffix of m/r.  Device-wide
// scan in three deterministic passes: per-tile sums, a one-block scan of the
// tile sums (forward for M, backward for S), and a per-tile apply that adds
// the carries to in-tile scans.  HBM-bound: reads r and m, writes the
// orbit table ((r, Phi) and (M, S) per star plus the sampled search levels)
// and, for the standalone call, the state's phi, mcum, ssuf.
#include "cmc_internal.hpp"

namespace cmc {
namespace {

constexpr int PT = kBlock;
constexpr int PJ = kPotTile / kBlock;  // 8 consecutive stars per thread

template <typename MT>
__global__ __launch_bounds__(PT) void k_pot_tile_sums(const double *__restrict__ r,
                                                      const MT *__restrict__ m,
                                                      const cmc_scalars *__restrict__ sc,
                                                      double *__restrict__ tsum,
                                                      int64_t tiles) {
  __shared__ double sh[PT / 64];
  const int64_t n = sc->n;
  const int64_t t = blockIdx.x;
  const int64_t base = t * kPotTile + static_cast<int64_t>(threadIdx.x) * PJ;
  double sm = 0.0, sq = 0.0;
#pragma unroll
  for (int j = 0; j < PJ; ++j) {
    const int64_t k = base + j;
    if (k < n) {
      const double mk = load_mass(m, k);
      sm += mk;
      sq += mk / r[k];
    }
  }
  const double tm = block_sum<PT>(sm, sh);
  const double tq = block_sum<PT>(sq, sh);
  if (threadIdx.x == 0) {
    tsum[t] = tm;
    tsum[tiles + t] = tq;
  }
}

constexpr int ST = 1024;

__global__ __launch_bounds__(ST) void k_pot_tile_scan(const double *__restrict__ tsum,
                                                      double *__restrict__ carry,
                                                      int64_t tiles) {
  __shared__ double sh[ST / 64];
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

template <typename MT, bool PUBLIC>
__global__ __launch_bounds__(PT) void k_pot_apply(const double *__restrict__ r,
                                                  const MT *__restrict__ m,
                                                  const cmc_scalars *__restrict__ sc,
                                                  const double *__restrict__ carry,
                                                  int64_t tiles, double *__restrict__ phi,
                                                  double *__restrict__ mcum,
                                                  double *__restrict__ ssuf, Levels lv,
                                                  MS *__restrict__ ms) {
  __shared__ double sh[PT / 64];
  const int64_t n = sc->n;
  const int64_t t = blockIdx.x;
  const int64_t base = t * kPotTile + static_cast<int64_t>(threadIdx.x) * PJ;
  double rr[PJ], pm[PJ], sq[PJ];
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < PJ; ++j) {
    const int64_t k = base + j;
    const bool ok = k < n;
    rr[j] = ok ? r[k] : 1.0;
    const double mk = ok ? load_mass(m, k) : 0.0;
    acc += mk;
    pm[j] = acc;  // inclusive prefix inside the thread
    sq[j] = mk / rr[j];
  }
  const double tm = acc;
  acc = 0.0;
#pragma unroll
  for (int j = PJ - 1; j >= 0; --j) {  // exclusive suffix inside the thread
    const double q = sq[j];
    sq[j] = acc;
    acc += q;
  }
  const double tq = acc;
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
        mcum[k] = M;
        ssuf[k] = S;
        phi[k] = ph;
      }
      put_table(lv, ms, k, rr[j], ph, M, S);
    }
  }
}

template <typename MT>
hipError_t run(const cmc_state &s, const Workspace &w, bool pub, hipStream_t st) {
  const MT *m = static_cast<const MT *>(s.m);
  const int64_t tiles = w.pot_tiles;
  const dim3 grid(static_cast<unsigned>(tiles));
  k_pot_tile_sums<MT><<<grid, PT, 0, st>>>(s.r, m, s.sc, w.pot_tsum, tiles);
  k_pot_tile_scan<<<1, ST, 0, st>>>(w.pot_tsum, w.pot_carry, tiles);
  const Levels lv = levels_of(w);
  if (pub)
    k_pot_apply<MT, true><<<grid, PT, 0, st>>>(s.r, m, s.sc, w.pot_carry, tiles, s.phi,
                                                s.mcum, s.ssuf, lv, w.ms);
  else
    k_pot_apply<MT, false><<<grid, PT, 0, st>>>(s.r, m, s.sc, w.pot_carry, tiles, s.phi,
                                                 s.mcum, s.ssuf, lv, w.ms);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_potential(const cmc_state &s, const Workspace &w, int precision,
                            bool public_arrays, hipStream_t st) {
  (void)precision;
  return s.m_f32 ? run<float>(s, w, public_arrays, st) : run<double>(s, w, public_arrays, st);
}

}  // namespace cmc

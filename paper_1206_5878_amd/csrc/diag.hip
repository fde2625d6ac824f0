// diag.hip -- diagnostics of a sorted state (arXiv:1206.5878, Sec. 2.1 step 6
// diagnostics; energy check of Sec. 4): T = sum m v^2 / 2, W = sum m Phi / 2,
// E = T + W, virial ratio 2T/|W|, total mass and the radii enclosing 1%, 10%,
// 50% and 90% of it.  Raw Philox blocks for inspection live here too.
#include "cmc_internal.hpp"

namespace cmc {
namespace {

constexpr int NT = kBlock;

template <typename MT>
__global__ __launch_bounds__(NT) void k_diag(const double *__restrict__ vr,
                                             const double *__restrict__ vt,
                                             const MT *__restrict__ m,
                                             const double *__restrict__ phi,
                                             const cmc_scalars *__restrict__ sc,
                                             double *__restrict__ part) {
  __shared__ double sh[NT / 64];
  const int64_t n = sc->n;
  double t = 0.0, wv = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * NT) {
    const double mi = load_mass(m, i);
    t += 0.5 * mi * (vr[i] * vr[i] + vt[i] * vt[i]);
    wv += 0.5 * mi * phi[i];
  }
  t = block_sum<NT>(t, sh);
  wv = block_sum<NT>(wv, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = t;
    part[2 * blockIdx.x + 1] = wv;
  }
}

__global__ __launch_bounds__(NT) void k_diag_final(const double *__restrict__ part, int nblocks,
                                                   const double *__restrict__ r,
                                                   const double *__restrict__ mcum,
                                                   const cmc_scalars *__restrict__ sc,
                                                   double *__restrict__ out) {
  __shared__ double sh[NT / 64];
  double T = 0.0, W = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += NT) {
    T += part[2 * b];
    W += part[2 * b + 1];
  }
  T = block_sum<NT>(T, sh);
  W = block_sum<NT>(W, sh);
  if (threadIdx.x != 0) return;
  const int64_t n = sc->n;
  const double M = n > 0 ? mcum[n - 1] : 0.0;
  out[0] = T;
  out[1] = W;
  out[2] = T + W;
  out[3] = W != 0.0 ? 2.0 * T / fabs(W) : 0.0;
  out[4] = M;
  const double fr[4] = {0.01, 0.1, 0.5, 0.9};
  for (int f = 0; f < 4; ++f) {
    // first k with mcum[k] >= f M
    int64_t lo = -1, hi = n;
    while (hi - lo > 1) {
      const int64_t mid = lo + ((hi - lo) >> 1);
      if (mcum[mid] >= fr[f] * M)
        hi = mid;
      else
        lo = mid;
    }
    out[5 + f] = hi < n ? r[hi] : __builtin_nan("");
  }
}

__global__ __launch_bounds__(NT) void k_philox(uint64_t key, const uint32_t *__restrict__ ctr,
                                               uint32_t *__restrict__ out, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
  if (i >= n) return;
  const U4 w = philox(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], key);
  out[4 * i] = w.x;
  out[4 * i + 1] = w.y;
  out[4 * i + 2] = w.z;
  out[4 * i + 3] = w.w;
}

template <typename MT>
hipError_t run(const cmc_state &s, const Workspace &w, double *out, hipStream_t st) {
  const int nb = static_cast<int>(w.star_blocks < kRedBlocks ? w.star_blocks : kRedBlocks);
  k_diag<MT><<<nb, NT, 0, st>>>(s.vr, s.vt, static_cast<const MT *>(s.m), s.phi, s.sc,
                                w.red_part);
  k_diag_final<<<1, NT, 0, st>>>(w.red_part, nb, s.r, s.mcum, s.sc, out);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_diagnostics(const cmc_state &s, const Workspace &w, double *out,
                              hipStream_t st) {
  return s.m_f32 ? run<float>(s, w, out, st) : run<double>(s, w, out, st);
}

hipError_t launch_philox(uint64_t key, const uint32_t *ctr, uint32_t *out, int64_t n,
                         hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_philox<<<static_cast<unsigned>(cdiv(n, NT)), NT, 0, st>>>(key, ctr, out, n);
  return hipGetLastError();
}

}  // namespace cmc

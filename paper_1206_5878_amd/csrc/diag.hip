// diag.hip -- diagnostics of a sorted state (arXiv:1206.5878, Sec. 2.1 step 6
// diagnostics; energy check and core-collapse runs of Sec. 4): T = sum m v^2 /
// 2, W = sum m Phi / 2, E = T + W, virial ratio 2T/|W|, total mass, the radii
// enclosing 1%, 10%, 50% and 90% of it, and the core: the density around each
// star from its radial neighbours (the 5 stars strictly inside a window of 7
// consecutive radii over the shell volume between its ends, after Casertano &
// Hut's 6th-order estimator), the core density sum rho^2 / sum rho and the
// density-weighted core radius sum rho r / sum rho.  Raw Philox blocks for
// inspection live here too.
#include "cmc_internal.hpp"

namespace cmc {
namespace {

constexpr int NT = kBlock;
constexpr int kDiagSums = 6;  // block partials of the diagnostics kernel

template <class Ctx, typename MT>
__global__ __launch_bounds__(NT) void k_diag(Ctx ctx) {
  __shared__ double sh[NT / 64];
  const ClusterArgs &A = ctx.args();
  const double *__restrict__ vr = A.s.vr;
  const double *__restrict__ vt = A.s.vt;
  const MT *__restrict__ m = static_cast<const MT *>(A.s.m);
  const double *__restrict__ phi = A.s.phi;
  const double *__restrict__ r = A.s.r;
  const int64_t n = A.s.sc->n;
  const int64_t blk = ctx.block();
  // T, W, sum rho, sum rho^2, sum rho r, windows used
  double v[kDiagSums] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t i = blk * NT + threadIdx.x; i < n; i += ctx.nblocks() * NT) {
    const double mi = load_mass(m, i);
    v[0] += 0.5 * mi * (vr[i] * vr[i] + vt[i] * vt[i]);
    v[1] += 0.5 * mi * phi[i];
    if (n >= 7) {
      int64_t a = i - 3;
      a = a < 0 ? 0 : (a > n - 7 ? n - 7 : a);
      const double lo = r[a], hi = r[a + 6];
      const double vol = (4.0 * kPi / 3.0) * (hi - lo) * (hi * hi + hi * lo + lo * lo);
      if (vol > 0.0) {
        double inner = 0.0;
#pragma unroll
        for (int q = 1; q <= 5; ++q) inner += load_mass(m, a + q);
        const double rho = inner / vol;
        v[2] += rho;
        v[3] += rho * rho;
        v[4] += rho * r[i];
        v[5] += 1.0;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kDiagSums; ++q) v[q] = block_sum<NT>(v[q], sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < kDiagSums; ++q) A.w.red_part[kDiagSums * blk + q] = v[q];
}

// One block per cluster; cluster c writes out[CMC_DIAG_N c .. CMC_DIAG_N c +
// CMC_DIAG_N - 1].
template <class Ctx>
__global__ __launch_bounds__(NT) void k_diag_final(Ctx ctx, double *__restrict__ out_all) {
  __shared__ double sh[NT / 64];
  const ClusterArgs &A = ctx.args();
  const double *__restrict__ part = A.w.red_part;
  const int64_t nblocks = blocks_of(kShDiag, A.w, A.s.cap);
  const double *__restrict__ r = A.s.r;
  const double *__restrict__ mcum = A.s.mcum;
  double *__restrict__ out = out_all + CMC_DIAG_N * ctx.index();
  double v[kDiagSums] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t b = threadIdx.x; b < nblocks; b += NT)
#pragma unroll
    for (int q = 0; q < kDiagSums; ++q) v[q] += part[kDiagSums * b + q];
#pragma unroll
  for (int q = 0; q < kDiagSums; ++q) v[q] = block_sum<NT>(v[q], sh);
  if (threadIdx.x != 0) return;
  const double T = v[0], W = v[1];
  const bool core = v[5] > 0.0 && v[2] > 0.0;
  out[9] = core ? v[4] / v[2] : __builtin_nan("");
  out[10] = core ? v[3] / v[2] : __builtin_nan("");
  const int64_t n = A.s.sc->n;
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

}  // namespace

hipError_t launch_diagnostics(const Target &t, bool m_f32, double *out, hipStream_t st) {
  return dispatch(t, [&](const auto &l) {
    using C = decltype(l.ctx(kShDiag));
    if (m_f32)
      k_diag<C, float><<<l.grid(kShDiag), NT, 0, st>>>(l.ctx(kShDiag));
    else
      k_diag<C, double><<<l.grid(kShDiag), NT, 0, st>>>(l.ctx(kShDiag));
    k_diag_final<<<l.grid(kShOne), NT, 0, st>>>(l.ctx(kShOne), out);
    return hipGetLastError();
  });
}

hipError_t launch_philox(uint64_t key, const uint32_t *ctr, uint32_t *out, int64_t n,
                         hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_philox<<<static_cast<unsigned>(cdiv(n, NT)), NT, 0, st>>>(key, ctr, out, n);
  return hipGetLastError();
}

}  // namespace cmc

// diag.hip -- diagnostics of a sorted state (arXiv:1206.5878, Sec. 2.1 step 6
// diagnostics; energy check of Sec. 4): T = sum m v^2 / 2, W = sum m Phi / 2,
// E = T + W, virial ratio 2T/|W|, total mass and the radii enclosing 1%, 10%,
// 50% and 90% of it.  Raw Philox blocks for inspection live here too.
#include "cmc_internal.hpp"

namespace cmc {
namespace {

constexpr int NT = kBlock;

template <class Ctx, typename MT>
__global__ __launch_bounds__(NT) void k_diag(Ctx ctx) {
  __shared__ double sh[NT / 64];
  const ClusterArgs &A = ctx.args();
  const double *__restrict__ vr = A.s.vr;
  const double *__restrict__ vt = A.s.vt;
  const MT *__restrict__ m = static_cast<const MT *>(A.s.m);
  const double *__restrict__ phi = A.s.phi;
  const int64_t n = A.s.sc->n;
  const int64_t blk = ctx.block();
  double t = 0.0, wv = 0.0;
  for (int64_t i = blk * NT + threadIdx.x; i < n; i += ctx.nblocks() * NT) {
    const double mi = load_mass(m, i);
    t += 0.5 * mi * (vr[i] * vr[i] + vt[i] * vt[i]);
    wv += 0.5 * mi * phi[i];
  }
  t = block_sum<NT>(t, sh);
  wv = block_sum<NT>(wv, sh);
  if (threadIdx.x == 0) {
    A.w.red_part[2 * blk] = t;
    A.w.red_part[2 * blk + 1] = wv;
  }
}

// One block per cluster; cluster c writes out[9 c .. 9 c + 8].
template <class Ctx>
__global__ __launch_bounds__(NT) void k_diag_final(Ctx ctx, double *__restrict__ out_all) {
  __shared__ double sh[NT / 64];
  const ClusterArgs &A = ctx.args();
  const double *__restrict__ part = A.w.red_part;
  const int64_t nblocks = blocks_of(kShDiag, A.w, A.s.cap);
  const double *__restrict__ r = A.s.r;
  const double *__restrict__ mcum = A.s.mcum;
  double *__restrict__ out = out_all + 9 * ctx.index();
  double T = 0.0, W = 0.0;
  for (int64_t b = threadIdx.x; b < nblocks; b += NT) {
    T += part[2 * b];
    W += part[2 * b + 1];
  }
  T = block_sum<NT>(T, sh);
  W = block_sum<NT>(W, sh);
  if (threadIdx.x != 0) return;
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

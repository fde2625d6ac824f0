// rindex.hip -- bucket index over the sorted radii, so that "the interval
// holding radius x" (the last k with r_k <= x, which selects the potential
// -(M_k / x + S_k) of Sec. 2.1 step 1 at a trial radius of step 5) costs one
// bucket read and one short scan instead of a search over the whole table.
//
// start[b] = the number of stars in buckets below b.  With b_k the bucket of
// r_k, that is k for every bucket b_(k-1) < b <= b_k: star k's thread writes
// its own range, so every entry is written once, in one pass over the radii
// with no clear and no scan.  Ranges longer than kRxShort (sparse radii,
// where a gap spans many buckets) go to a list, in pieces of at most
// kRxPiece, which a second pass fills block by block; that pass also fills
// the buckets above the last star's with n.
#include <algorithm>

#include "cmc_internal.hpp"

namespace cmc {
namespace {

constexpr int NT = kBlock;

// One thread per cluster.
template <class Ctx>
__global__ void k_rindex_prep(Ctx ctx) {
  const ClusterArgs &A = ctx.args();
  const double *__restrict__ r = A.s.r;
  const int lg_nb = A.w.rx_lg_nb;
  RIndexCtl *__restrict__ ctl = A.w.rx_ctl;
  const int64_t n = A.s.sc->n;
  RIndexCtl c{0ull, 0ull, 0u, static_cast<uint32_t>(n > 0 ? n : 0)};
  if (n > 0) {
    c.lo = rbits(r[0]);
    c.hi = rbits(r[n - 1]);
    const uint64_t range = c.hi > c.lo ? c.hi - c.lo : 0ull;
    const int bits = range ? 64 - __clzll(static_cast<long long>(range)) : 0;
    c.shift = static_cast<uint32_t>(bits > lg_nb ? bits - lg_nb : 0);
  }
  *ctl = c;
  *A.w.rx_nlong = 0u;
}

// Bucket of a table radius; clamped to [lo, hi] so that a table that is not
// sorted gives a wrong index rather than a write out of bounds.
__device__ __forceinline__ int64_t bucket(double x, const RIndexCtl &c) {
  uint64_t k = rbits(x);
  k = k < c.lo ? c.lo : (k > c.hi ? c.hi : k);
  return static_cast<int64_t>((k - c.lo) >> c.shift);
}

// Bucket of the last star (its radius's bits are hi); -1 for no star.
__device__ __forceinline__ int64_t last_bucket(const RIndexCtl &c) {
  return c.n > 0 ? static_cast<int64_t>((c.hi - c.lo) >> c.shift) : -1;
}

template <class Ctx>
__global__ __launch_bounds__(NT) void k_rindex_fill(Ctx ctx) {
  const ClusterArgs &A = ctx.args();
  const double *__restrict__ r = A.s.r;
  uint32_t *__restrict__ start = A.w.rx_start;
  const RIndexCtl c = *A.w.rx_ctl;
  const int64_t n = c.n;
  const int64_t k = ctx.block() * NT + threadIdx.x;
  // buckets [b0, b1) take k
  int64_t b0 = 0, b1 = 0;
  if (k < n) {
    b0 = k > 0 ? bucket(r[k - 1], c) + 1 : 0;
    b1 = bucket(r[k], c) + 1;
  }
  const int64_t len = b1 - b0;
  if (len > 0 && len <= kRxShort)
    for (int64_t b = b0; b < b1; ++b) start[b] = static_cast<uint32_t>(k);
  // the long ranges: one list slot per piece, one atomic per wavefront
  const uint32_t pieces = len > kRxShort ? static_cast<uint32_t>(cdiv(len, kRxPiece)) : 0u;
  if (__ballot(pieces != 0u) == 0ull) return;  // wave-uniform
  const uint32_t incl = wave_incl_scan(pieces);
  const uint32_t total = __shfl(incl, 63, 64);
  uint32_t base = 0u;
  if ((threadIdx.x & 63) == 63) base = atomicAdd(A.w.rx_nlong, total);
  base = __shfl(base, 63, 64);
  const int64_t e0 = static_cast<int64_t>(base) + (incl - pieces);
  for (uint32_t q = 0; q < pieces && e0 + q < A.w.rx_long_cap; ++q) {
    const int64_t a = b0 + static_cast<int64_t>(q) * kRxPiece;
    const int64_t e = a + kRxPiece < b1 ? a + kRxPiece : b1;
    A.w.rx_long[e0 + q] =
        RxRange{static_cast<uint32_t>(a), static_cast<uint32_t>(e), static_cast<uint32_t>(k), 0u};
  }
}

// Block j fills the listed ranges j, j + grid, ...; then the grid fills the
// buckets above the last star's with n.
template <class Ctx>
__global__ __launch_bounds__(NT) void k_rindex_long(Ctx ctx) {
  const ClusterArgs &A = ctx.args();
  const RIndexCtl c = *A.w.rx_ctl;
  const int64_t cnt0 = *A.w.rx_nlong;
  const int64_t cnt = cnt0 < A.w.rx_long_cap ? cnt0 : A.w.rx_long_cap;
  uint32_t *__restrict__ start = A.w.rx_start;
  for (int64_t e = ctx.block(); e < cnt; e += ctx.nblocks()) {
    const RxRange g = A.w.rx_long[e];
    for (int64_t b = g.b0 + threadIdx.x; b < g.b1; b += NT) start[b] = g.k;
  }
  const uint32_t nn = static_cast<uint32_t>(c.n);
  for (int64_t b = last_bucket(c) + 1 + ctx.block() * NT + threadIdx.x; b <= A.w.rx_nb;
       b += ctx.nblocks() * NT)
    start[b] = nn;
}

}  // namespace

hipError_t launch_rindex(const Target &t, hipStream_t st) {
  return dispatch(t, [&](const auto &l) {
    k_rindex_prep<<<l.grid(kShOne), 1, 0, st>>>(l.ctx(kShOne));
    k_rindex_fill<<<l.grid(kShRxFill), NT, 0, st>>>(l.ctx(kShRxFill));
    k_rindex_long<<<l.grid(kShRxLong), NT, 0, st>>>(l.ctx(kShRxLong));
    return hipGetLastError();
  });
}

}  // namespace cmc

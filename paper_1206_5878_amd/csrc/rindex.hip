// rindex.hip -- bucket index over the sorted radii, so that "the interval
// holding radius x" (the last k with r_k <= x, which selects the potential
// -(M_k / x + S_k) of Sec. 2.1 step 1 at a trial radius of step 5) costs one
// bucket read and one short scan instead of a search over the whole table.
//
// Built in three streaming passes: clear start[]; the last star of every
// non-empty bucket b writes its index + 1 into start[b + 1]; an inclusive
// prefix maximum over start[] then fills every bucket with the number of
// stars in the buckets before it (empty buckets included).
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
}

// Bucket of a table radius; clamped to [lo, hi] so that a table that is not
// sorted gives a wrong index rather than a write out of bounds.
__device__ __forceinline__ int64_t bucket(double x, const RIndexCtl &c) {
  uint64_t k = rbits(x);
  k = k < c.lo ? c.lo : (k > c.hi ? c.hi : k);
  return static_cast<int64_t>((k - c.lo) >> c.shift);
}

constexpr int kScanTile = NT * 16;
static_assert(kScanTile == kRxTile, "prefix-maximum tile");

template <class Ctx>
__global__ __launch_bounds__(NT) void k_rindex_clear(Ctx ctx) {
  const ClusterArgs &A = ctx.args();
  uint32_t *__restrict__ start = A.w.rx_start;
  const int64_t len = A.w.rx_nb + 1;
  for (int64_t b = ctx.block() * NT + threadIdx.x; b < len; b += ctx.nblocks() * NT)
    start[b] = 0u;
}

template <class Ctx>
__global__ __launch_bounds__(NT) void k_rindex_ends(Ctx ctx) {
  const ClusterArgs &A = ctx.args();
  const double *__restrict__ r = A.s.r;
  uint32_t *__restrict__ start = A.w.rx_start;
  const RIndexCtl c = *A.w.rx_ctl;
  const int64_t n = c.n;
  for (int64_t k = ctx.block() * NT + threadIdx.x; k < n; k += ctx.nblocks() * NT) {
    const int64_t bk = bucket(r[k], c);
    if (k == n - 1 || bucket(r[k + 1], c) != bk) start[bk + 1] = static_cast<uint32_t>(k + 1);
  }
}

__device__ __forceinline__ uint32_t wave_incl_max(uint32_t v) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t u = __shfl_up(v, o, 64);
    if (l >= o) v = u > v ? u : v;
  }
  return v;
}

// Exclusive prefix maximum over the block's threads (0 for thread 0).
__device__ __forceinline__ uint32_t block_excl_max(uint32_t v, uint32_t *sh) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t inc = wave_incl_max(v);
  uint32_t exc = __shfl_up(inc, 1, 64);
  if (l == 0) exc = 0u;
  if (l == 63) sh[w] = inc;
  __syncthreads();
  uint32_t base = 0u;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i)
    if (i < w) base = sh[i] > base ? sh[i] : base;
  __syncthreads();
  return base > exc ? base : exc;
}

template <class Ctx>
__global__ __launch_bounds__(NT) void k_rindex_tilemax(Ctx ctx) {
  __shared__ uint32_t sh[NT / 64];
  const ClusterArgs &A = ctx.args();
  const uint32_t *__restrict__ start = A.w.rx_start;
  const int64_t len = A.w.rx_nb + 1;
  uint32_t *__restrict__ tmax = A.w.rx_tile;
  const int64_t blk = ctx.block();
  const int64_t base = blk * kScanTile;
  uint32_t v = 0u;
  for (int j = 0; j < 16; ++j) {
    const int64_t b = base + j * NT + threadIdx.x;
    if (b < len) v = start[b] > v ? start[b] : v;
  }
  v = wave_incl_max(v);
  if ((threadIdx.x & 63) == 63) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t m = 0u;
    for (int i = 0; i < NT / 64; ++i) m = sh[i] > m ? sh[i] : m;
    tmax[blk] = m;
  }
}

// One block per cluster: exclusive prefix maximum over the tile maxima, in
// place.
template <class Ctx>
__global__ __launch_bounds__(NT) void k_rindex_tilescan(Ctx ctx) {
  __shared__ uint32_t sh[NT / 64];
  const ClusterArgs &A = ctx.args();
  uint32_t *__restrict__ tmax = A.w.rx_tile;
  const int64_t tiles = cdiv(A.w.rx_nb + 1, kScanTile);
  __shared__ uint32_t blk;
  uint32_t carry = 0u;
  for (int64_t t0 = 0; t0 < tiles; t0 += NT) {
    const int64_t t = t0 + threadIdx.x;
    const uint32_t v = t < tiles ? tmax[t] : 0u;
    const uint32_t ex = block_excl_max(v, sh);
    if (t < tiles) tmax[t] = carry > ex ? carry : ex;
    if (threadIdx.x == NT - 1) blk = ex > v ? ex : v;
    __syncthreads();
    carry = blk > carry ? blk : carry;
    __syncthreads();
  }
}

template <class Ctx>
__global__ __launch_bounds__(NT) void k_rindex_apply(Ctx ctx) {
  __shared__ uint32_t sh[NT / 64];
  const ClusterArgs &A = ctx.args();
  uint32_t *__restrict__ start = A.w.rx_start;
  const int64_t len = A.w.rx_nb + 1;
  const uint32_t *__restrict__ tcarry = A.w.rx_tile;
  const int64_t blk = ctx.block();
  const int64_t base = blk * kScanTile + threadIdx.x * 16;
  // 16 consecutive entries per thread, moved as four 16-byte vectors where
  // the whole vector is in range (start[] is 256-byte aligned)
  uint32_t v[16];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t b = base + 4 * q;
    if (b + 4 <= len) {
      const uint4 x = *reinterpret_cast<const uint4 *>(start + b);
      v[4 * q] = x.x;
      v[4 * q + 1] = x.y;
      v[4 * q + 2] = x.z;
      v[4 * q + 3] = x.w;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) v[4 * q + j] = (b + j < len) ? start[b + j] : 0u;
    }
  }
  uint32_t run = 0u;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    run = v[j] > run ? v[j] : run;
    v[j] = run;
  }
  uint32_t ex = block_excl_max(run, sh);
  const uint32_t c = tcarry[blk];
  ex = c > ex ? c : ex;
#pragma unroll
  for (int j = 0; j < 16; ++j) v[j] = ex > v[j] ? ex : v[j];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t b = base + 4 * q;
    if (b + 4 <= len) {
      *reinterpret_cast<uint4 *>(start + b) =
          make_uint4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (b + j < len) start[b + j] = v[4 * q + j];
    }
  }
}

}  // namespace

hipError_t launch_rindex(const Target &t, hipStream_t st) {
  return dispatch(t, [&](const auto &l) {
    k_rindex_prep<<<l.grid(kShOne), 1, 0, st>>>(l.ctx(kShOne));
    k_rindex_clear<<<l.grid(kShRxClear), NT, 0, st>>>(l.ctx(kShRxClear));
    k_rindex_ends<<<l.grid(kShDiag), NT, 0, st>>>(l.ctx(kShDiag));
    k_rindex_tilemax<<<l.grid(kShRxTile), NT, 0, st>>>(l.ctx(kShRxTile));
    k_rindex_tilescan<<<l.grid(kShOne), NT, 0, st>>>(l.ctx(kShOne));
    k_rindex_apply<<<l.grid(kShRxTile), NT, 0, st>>>(l.ctx(kShRxTile));
    return hipGetLastError();
  });
}

}  // namespace cmc

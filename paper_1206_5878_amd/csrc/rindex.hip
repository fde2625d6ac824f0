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

__global__ void k_rindex_prep(const double *__restrict__ r, const cmc_scalars *__restrict__ sc,
                              int lg_nb, RIndexCtl *__restrict__ ctl) {
  const int64_t n = sc->n;
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

__global__ __launch_bounds__(NT) void k_rindex_clear(uint32_t *__restrict__ start, int64_t len) {
  for (int64_t b = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; b < len;
       b += static_cast<int64_t>(gridDim.x) * NT)
    start[b] = 0u;
}

__global__ __launch_bounds__(NT) void k_rindex_ends(const double *__restrict__ r,
                                                    const RIndexCtl *__restrict__ ctl,
                                                    uint32_t *__restrict__ start) {
  const RIndexCtl c = *ctl;
  const int64_t n = c.n;
  const int64_t k = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
  if (k >= n) return;
  const int64_t bk = bucket(r[k], c);
  if (k == n - 1 || bucket(r[k + 1], c) != bk) start[bk + 1] = static_cast<uint32_t>(k + 1);
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

__global__ __launch_bounds__(NT) void k_rindex_tilemax(const uint32_t *__restrict__ start,
                                                       int64_t len, uint32_t *__restrict__ tmax) {
  __shared__ uint32_t sh[NT / 64];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
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
    tmax[blockIdx.x] = m;
  }
}

// One block: exclusive prefix maximum over the tile maxima, in place.
__global__ __launch_bounds__(NT) void k_rindex_tilescan(uint32_t *__restrict__ tmax,
                                                        int64_t tiles) {
  __shared__ uint32_t sh[NT / 64];
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

__global__ __launch_bounds__(NT) void k_rindex_apply(uint32_t *__restrict__ start, int64_t len,
                                                     const uint32_t *__restrict__ tcarry) {
  __shared__ uint32_t sh[NT / 64];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * 16;
  uint32_t v[16];
  uint32_t run = 0u;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    v[j] = (base + j < len) ? start[base + j] : 0u;
    run = v[j] > run ? v[j] : run;
    v[j] = run;
  }
  uint32_t ex = block_excl_max(run, sh);
  const uint32_t c = tcarry[blockIdx.x];
  ex = c > ex ? c : ex;
#pragma unroll
  for (int j = 0; j < 16; ++j)
    if (base + j < len) start[base + j] = ex > v[j] ? ex : v[j];
}

}  // namespace

hipError_t launch_rindex(const cmc_state &s, const Workspace &w, hipStream_t st) {
  const int64_t len = w.rx_nb + 1;
  const int64_t tiles = cdiv(len, kScanTile);
  k_rindex_prep<<<1, 1, 0, st>>>(s.r, s.sc, w.rx_lg_nb, w.rx_ctl);
  k_rindex_clear<<<static_cast<unsigned>(std::min<int64_t>(cdiv(len, NT), 4096)), NT, 0, st>>>(
      w.rx_start, len);
  k_rindex_ends<<<static_cast<unsigned>(w.star_blocks), NT, 0, st>>>(s.r, w.rx_ctl, w.rx_start);
  k_rindex_tilemax<<<static_cast<unsigned>(tiles), NT, 0, st>>>(w.rx_start, len, w.rx_tile);
  k_rindex_tilescan<<<1, NT, 0, st>>>(w.rx_tile, tiles);
  k_rindex_apply<<<static_cast<unsigned>(tiles), NT, 0, st>>>(w.rx_start, len, w.rx_tile);
  return hipGetLastError();
}

}  // namespace cmc

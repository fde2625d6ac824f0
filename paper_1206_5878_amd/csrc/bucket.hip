// bucket.hip -- the step's radial sort (arXiv:1206.5878, Sec. 2.1 step 6) by
// the positions the orbit pass already found.  For each staged star the
// orbit pass stored c = the number of old sorted radii <= r_new.  c is
// monotone in r_new, so the sort is a counting sort on c followed by a
// comparison sort of each run of equal c:
//   1. per tile of 16384 stars, an LDS histogram over buckets of 2048
//      consecutive values of c (escapers in a bin of their own);
//   2. per bucket, exclusive offsets of the tiles (column scan), and per
//      cluster the bucket starts (the escapers' bin last: they are dropped);
//   3. per tile, a scatter of 16-byte entries (radius key, staged index,
//      c mod 2048) to their bucket;
//   4. per bucket, one block: a counting sort on c mod 2048 in LDS (16-bit
//      counters, two to a word), each run of equal c (about one star) sorted
//      by (radius, staged index), then the staged records gathered in that
//      order into the state arrays.
// The result is the stable sort of the staged stars by radius, the same
// permutation as the radix sort.  Records move once (one random read each,
// a whole line for the 32-byte records of f32 masses); entries move once.
// A bucket has 2048 stars on average: one that holds more than 4096 (a state
// far from the old one, or many equal radii) is merge-sorted by its block in
// global memory instead, and a run of more than 48 equal c by a bitonic
// network.
#include <type_traits>

#include "cmc_internal.hpp"

namespace cmc {
namespace {

constexpr int HT = 1024;      // threads of the tile and scan kernels
constexpr int BT = 512;       // threads of a bucket's sort
constexpr int kSubMax = 48;   // longest run of equal c sorted by insertion
constexpr int kMergeRun = 16; // outputs per thread of a merge step

__device__ __forceinline__ int64_t buckets_of(int64_t n) { return (n >> kBucketShift) + 1; }

// Bin of a staged star among nb buckets of kept stars and the escapers' bin
// nb (c <= n always; the clamp only keeps LDS indices in range).
__device__ __forceinline__ uint32_t bin_of(uint32_t c, int64_t nb) {
  if (c == kBucketEsc) return static_cast<uint32_t>(nb);
  const uint32_t b = c >> kBucketShift;
  return b < nb ? b : static_cast<uint32_t>(nb - 1);
}

// Order of the sort: radius bits, then staged index (both unique together).
__device__ __forceinline__ bool before(uint64_t ka, uint32_t ia, uint64_t kb, uint32_t ib) {
  return ka < kb || (ka == kb && ia < ib);
}

template <class Ctx>
__global__ __launch_bounds__(HT) void k_bkt_hist(Ctx ctx) {
  __shared__ uint32_t hist[kBucketBins];
  const ClusterArgs &A = ctx.args();
  const int64_t n = A.s.sc->n;
  const int64_t t = ctx.block();
  const int64_t k0 = t * kBucketTile;
  if (k0 >= n) return;
  const int64_t nb = buckets_of(n);
  const int bins = static_cast<int>(nb + 1);
  const uint32_t *__restrict__ bkey = A.w.bkey;
  for (int b = threadIdx.x; b < bins; b += HT) hist[b] = 0u;
  __syncthreads();
  const int64_t k1 = k0 + kBucketTile < n ? k0 + kBucketTile : n;
#pragma unroll 8
  for (int j = 0; j < kBucketTile / HT; ++j) {
    const int64_t k = k0 + j * HT + threadIdx.x;
    if (k < k1) {
      atomicAdd(&hist[bin_of(bkey[k], nb)], 1u);
    }
  }
  __syncthreads();
  uint32_t *__restrict__ row = A.w.bkt_cnt + t * A.w.bkt_bins;
  for (int b = threadIdx.x; b < bins; b += HT) row[b] = hist[b];
}

// Block g: bins kBktColGroup g .. kBktColGroup (g + 1) - 1.  Counts become tile
// offsets inside the bin; tot gets the bin sums.
template <class Ctx>
__global__ __launch_bounds__(HT) void k_bkt_colscan(Ctx ctx) {
  const ClusterArgs &A = ctx.args();
  const int64_t n = A.s.sc->n;
  const int64_t bins = buckets_of(n) + 1;
  const int64_t c0 = ctx.block() * kBktColGroup;
  if (c0 >= bins) return;  // block-uniform
  column_scan<HT, kBktColGroup>(A.w.bkt_cnt, A.w.bkt_bins, cdiv(n, kBucketTile), c0, bins, A.w.bkt_tot);
}

// One block per cluster: bucket starts; the escapers' bin comes last, so the
// kept stars are the first start[nb].  The state's n becomes that count, and
// the energy correction of the staged stars is left pending (corr) or none.
template <class Ctx>
__global__ __launch_bounds__(HT) void k_bkt_start(Ctx ctx, int corr) {
  __shared__ uint32_t sh[HT / 64];
  const ClusterArgs &A = ctx.args();
  cmc_scalars *__restrict__ sc = A.s.sc;
  const uint32_t *__restrict__ tot = A.w.bkt_tot;
  uint32_t *__restrict__ start = A.w.bkt_start;
  const int64_t n = sc->n;  // read by every thread before the scans' barriers
  const int64_t nb = buckets_of(n);
  uint32_t carry = 0u;
  for (int64_t b0 = 0; b0 <= nb; b0 += HT) {
    const int64_t b = b0 + threadIdx.x;
    const uint32_t v = b <= nb ? tot[b] : 0u;
    uint32_t all;
    const uint32_t ex = block_excl_scan<HT>(v, sh, &all);
    if (b <= nb) start[b] = carry + ex;
    carry += all;
  }
  if (threadIdx.x == 0) {
    start[nb + 1] = carry;
    const int64_t kept = n - static_cast<int64_t>(tot[nb]);
    A.w.bkt_info[0] = n;
    A.w.bkt_info[1] = kept;
    sc->n = kept;
    sc->corr_n = corr ? n : 0;
  }
}

// Entries to their buckets at LDS-atomic slots.
template <class Ctx>
__global__ __launch_bounds__(HT) void k_bkt_scatter(Ctx ctx) {
  __shared__ uint32_t cur[kBucketBins];
  const ClusterArgs &A = ctx.args();
  const int64_t n = A.w.bkt_info[0];
  // Consecutive tiles on one XCD (blocks go round-robin over the 8 XCDs):
  // their runs of a bucket are adjacent, so partial lines meet in one L2.
  int64_t t = ctx.block();
  {
    const int64_t q = ctx.nblocks() / 8;
    if (t < 8 * q) t = (t % 8) * q + t / 8;
  }
  const int64_t k0 = t * kBucketTile;
  if (k0 >= n) return;
  const int64_t nb = buckets_of(n);
  const uint32_t *__restrict__ row = A.w.bkt_cnt + t * A.w.bkt_bins;
  const uint32_t *__restrict__ start = A.w.bkt_start;
  const uint32_t *__restrict__ bkey = A.w.bkey;
  const uint64_t *__restrict__ keys = A.w.keys[0];
  BktEnt *__restrict__ bent = A.w.bent;
  for (int b = threadIdx.x; b < nb; b += HT) cur[b] = start[b] + row[b];
  __syncthreads();
  const int64_t k1 = k0 + kBucketTile < n ? k0 + kBucketTile : n;
#pragma unroll 4
  for (int j = 0; j < kBucketTile / HT; ++j) {
    const int64_t k = k0 + j * HT + threadIdx.x;
    if (k < k1) {
      const uint32_t c = bkey[k];
      if (c != kBucketEsc) {
        const uint32_t pos = atomicAdd(&cur[bin_of(c, nb)], 1u);
        BktEnt e;
        e.key = keys[k];
        e.idx = static_cast<uint32_t>(k);
        e.sub = c & (kBucketSpan - 1);
        bent[pos] = e;
      }
    }
  }
}

template <typename MT>
__device__ __forceinline__ void put_star(const ClusterArgs &A, int64_t p, const StageRec<MT> &rec) {
  A.s.r[p] = rec.r;
  A.s.vr[p] = rec.vr;
  A.s.vt[p] = rec.vt;
  static_cast<MT *>(A.s.m)[p] = rec.m;
  A.s.id[p] = rec.id;
}

// Bitonic sort of the first `count` entries (count <= kBucketSortCap) of
// (K, V) by (K, V); ends with a barrier.
__device__ void bitonic_lds(uint64_t *K, uint32_t *V, int count) {
  int P = 1;
  while (P < count) P <<= 1;
  for (int p = count + threadIdx.x; p < P; p += BT) {
    K[p] = ~0ull;
    V[p] = ~0u;
  }
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int x = threadIdx.x; x < P / 2; x += BT) {
        const int i = 2 * x - (x & (j - 1));
        const int l = i + j;
        const uint64_t ki = K[i], kl = K[l];
        const uint32_t vi = V[i], vl = V[l];
        const bool up = (i & k) == 0;
        if (before(kl, vl, ki, vi) == up) {
          K[i] = kl;
          K[l] = ki;
          V[i] = vl;
          V[l] = vi;
        }
      }
      __syncthreads();
    }
  }
}

// One merge step: sorted runs of width w of (sk, sv) pairwise into (dk, dv).
// Each thread finds where its kMergeRun outputs start in the two runs
// (a binary search along the merge path), then merges them in order.
__device__ void merge_step(const uint64_t *sk, const uint32_t *sv, uint64_t *dk, uint32_t *dv,
                           int64_t count, int64_t w) {
  for (int64_t d0 = static_cast<int64_t>(threadIdx.x) * kMergeRun; d0 < count;
       d0 += static_cast<int64_t>(BT) * kMergeRun) {
    const int64_t lo = d0 / (2 * w) * (2 * w);
    const int64_t a1 = lo + w < count ? lo + w : count;
    const int64_t b1 = lo + 2 * w < count ? lo + 2 * w : count;
    const int64_t na = a1 - lo, nbb = b1 - a1, dd = d0 - lo;
    int64_t x = dd - nbb > 0 ? dd - nbb : 0;
    int64_t y = dd < na ? dd : na;
    while (x < y) {
      const int64_t mid = (x + y) >> 1;
      const int64_t jb = a1 + dd - mid - 1;
      if (before(sk[lo + mid], sv[lo + mid], sk[jb], sv[jb]))
        x = mid + 1;
      else
        y = mid;
    }
    int64_t ia = lo + x, ib = a1 + dd - x;
    const int64_t e = d0 + kMergeRun < b1 ? d0 + kMergeRun : b1;
    for (int64_t d = d0; d < e; ++d) {
      const bool take_a = ib >= b1 || (ia < a1 && before(sk[ia], sv[ia], sk[ib], sv[ib]));
      const int64_t from = take_a ? ia++ : ib++;
      dk[d] = sk[from];
      dv[d] = sv[from];
    }
  }
}

// The staged records in the order of V's staged indices, into the state at
// out .. out + count (and, with corr, each star's staged index into perm; a
// state with LFSR113 streams takes each star's staged stream state along).
template <typename MT>
__device__ __forceinline__ void gather(const ClusterArgs &A, const uint32_t *V, int64_t out,
                                       int64_t count, int corr) {
  const StageRec<MT> *__restrict__ stage = static_cast<const StageRec<MT> *>(A.w.stage);
  constexpr int B = 8;  // records in flight per thread
  for (int64_t p0 = 0; p0 < count; p0 += B * BT) {
    StageRec<MT> rec[B];
    uint32_t src[B];
#pragma unroll
    for (int q = 0; q < B; ++q) {
      const int64_t p = p0 + q * BT + threadIdx.x;
      src[q] = 0u;
      if (p < count) {
        src[q] = V[p];
        rec[q] = stage[src[q]];
      }
    }
#pragma unroll
    for (int q = 0; q < B; ++q) {
      const int64_t p = p0 + q * BT + threadIdx.x;
      if (p < count) {
        put_star<MT>(A, out + p, rec[q]);
        if (corr) A.w.perm[out + p] = src[q];
        if (A.s.rng) store_lfsr(A.s.rng, out + p, A.w.rng_stage[src[q]]);
      }
    }
  }
}

// A bucket too large for LDS: its block sorts runs of kBucketSortCap in LDS,
// merges them in the radix sort's key buffers (at the bucket's own range, so
// buckets never overlap), then gathers the staged records in order.
template <typename MT>
__device__ void sort_large(const ClusterArgs &A, uint32_t base, int64_t count, uint64_t *K,
                           uint32_t *V, int corr) {
  uint64_t *kb[2] = {A.w.keys[0] + base, A.w.keys[1] + base};
  uint32_t *vb[2] = {A.w.vals[0] + base, A.w.vals[1] + base};
  const BktEnt *__restrict__ bent = A.w.bent + base;
  for (int64_t r0 = 0; r0 < count; r0 += kBucketSortCap) {
    const int m = static_cast<int>(count - r0 < kBucketSortCap ? count - r0 : kBucketSortCap);
    for (int s = threadIdx.x; s < m; s += BT) {
      const BktEnt e = bent[r0 + s];
      K[s] = e.key;
      V[s] = e.idx;
    }
    __syncthreads();
    bitonic_lds(K, V, m);
    for (int s = threadIdx.x; s < m; s += BT) {
      kb[0][r0 + s] = K[s];
      vb[0][r0 + s] = V[s];
    }
    __syncthreads();
  }
  int src = 0;
  for (int64_t w = kBucketSortCap; w < count; w <<= 1) {
    merge_step(kb[src], vb[src], kb[src ^ 1], vb[src ^ 1], count, w);
    __syncthreads();
    src ^= 1;
  }
  gather<MT>(A, vb[src], base, count, corr);
}

// One block per bucket.  sub: 16-bit counts, then starts, of each value of
// c mod 2048 (two to a word); entries (K radius key, V staged index) are
// placed by c, then each run of equal c is put in (K, V) order.
template <class Ctx, typename MT>
__global__ __launch_bounds__(BT) void k_bkt_sort(Ctx ctx, int corr) {
  __shared__ uint32_t sub[kBucketSpan / 2];
  __shared__ uint64_t K[kBucketSortCap];
  __shared__ uint32_t V[kBucketSortCap];
  __shared__ uint32_t sh[BT / 64];
  __shared__ int big;
  const ClusterArgs &A = ctx.args();
  const int64_t n = A.w.bkt_info[0];
  const int64_t b = ctx.block();
  if (b >= buckets_of(n)) return;
  const uint32_t base = A.w.bkt_start[b];
  const int64_t count = static_cast<int64_t>(A.w.bkt_start[b + 1]) - base;
  if (count <= 0) return;
  if (count > kBucketSortCap) {
    sort_large<MT>(A, base, count, K, V, corr);
    return;
  }
  const int cnt = static_cast<int>(count);
  const BktEnt *__restrict__ bent = A.w.bent + base;
  for (int q = threadIdx.x; q < kBucketSpan / 2; q += BT) sub[q] = 0u;
  if (threadIdx.x == 0) big = 0;
  __syncthreads();
  constexpr int PER = kBucketSortCap / BT;
  uint64_t ek[PER];
  uint32_t ev[PER], es[PER], rk[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int s = j * BT + threadIdx.x;
    ek[j] = 0ull;
    ev[j] = 0u;
    es[j] = 0u;
    rk[j] = 0u;
    if (s < cnt) {
      const BktEnt e = bent[s];
      ek[j] = e.key;
      ev[j] = e.idx;
      es[j] = e.sub & (kBucketSpan - 1);
      const uint32_t sh16 = (es[j] & 1u) * 16u;  // counts stay below 2^16: cnt <= 4096
      rk[j] = (atomicAdd(&sub[es[j] >> 1], 1u << sh16) >> sh16) & 0xFFFFu;
    }
  }
  __syncthreads();
  {
    constexpr int Q = kBucketSpan / 2 / BT;  // words of counts per thread
    uint32_t v[2 * Q], sum = 0u, mx = 0u;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const uint32_t wd = sub[threadIdx.x * Q + q];
      v[2 * q] = wd & 0xFFFFu;
      v[2 * q + 1] = wd >> 16;
    }
#pragma unroll
    for (int q = 0; q < 2 * Q; ++q) {
      sum += v[q];
      mx = v[q] > mx ? v[q] : mx;
    }
    if (mx > static_cast<uint32_t>(kSubMax)) big = 1;
    uint32_t acc = block_excl_scan<BT>(sum, sh, static_cast<uint32_t *>(nullptr));
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const uint32_t lo = acc, hi = acc + v[2 * q];
      sub[threadIdx.x * Q + q] = lo | (hi << 16);  // starts stay below 2^16 as well
      acc = hi + v[2 * q + 1];
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int s = j * BT + threadIdx.x;
    if (s < cnt) {
      const uint32_t p = ((sub[es[j] >> 1] >> ((es[j] & 1u) * 16u)) & 0xFFFFu) + rk[j];
      K[p] = ek[j];
      V[p] = ev[j];
    }
  }
  __syncthreads();
  if (!big) {
    for (int q = threadIdx.x; q < kBucketSpan; q += BT) {
      const int a = static_cast<int>((sub[q >> 1] >> ((q & 1) * 16)) & 0xFFFFu);
      const int e = q + 1 < kBucketSpan
                        ? static_cast<int>((sub[(q + 1) >> 1] >> (((q + 1) & 1) * 16)) & 0xFFFFu)
                        : cnt;
      for (int x = a + 1; x < e; ++x) {
        const uint64_t kx = K[x];
        const uint32_t vx = V[x];
        int y = x - 1;
        while (y >= a && before(kx, vx, K[y], V[y])) {
          K[y + 1] = K[y];
          V[y + 1] = V[y];
          --y;
        }
        K[y + 1] = kx;
        V[y + 1] = vx;
      }
    }
    __syncthreads();
  } else {
    bitonic_lds(K, V, cnt);
  }
  gather<MT>(A, V, base, cnt, corr);
}

template <class L, typename MT>
hipError_t run(const L &l, int corr, hipStream_t st) {
  k_bkt_hist<<<l.grid(kShBktTile), HT, 0, st>>>(l.ctx(kShBktTile));
  k_bkt_colscan<<<l.grid(kShBktGroup), HT, 0, st>>>(l.ctx(kShBktGroup));
  k_bkt_start<<<l.grid(kShOne), HT, 0, st>>>(l.ctx(kShOne), corr);
  k_bkt_scatter<<<l.grid(kShBktTile), HT, 0, st>>>(l.ctx(kShBktTile));
  k_bkt_sort<decltype(l.ctx(kShBktSort)), MT>
      <<<l.grid(kShBktSort), BT, 0, st>>>(l.ctx(kShBktSort), corr);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_bucket_sort(const Target &t, bool m_f32, bool corr, hipStream_t st) {
  const int c = corr ? 1 : 0;
  return dispatch(t, [&](const auto &l) {
    return m_f32 ? run<std::decay_t<decltype(l)>, float>(l, c, st)
                 : run<std::decay_t<decltype(l)>, double>(l, c, st);
  });
}

}  // namespace cmc

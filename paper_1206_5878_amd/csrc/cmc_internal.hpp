// cmc_internal.hpp -- device helpers and workspace layout shared by the HIP
// translation units of libcmc.so.  gfx950: 64-lane wavefronts.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/cmc.h"

namespace cmc {

constexpr double kPi = 3.14159265358979323846;
constexpr double kInf = __builtin_inf();
constexpr float kInfF = __builtin_inff();

// Philox counter word 2: what a draw is for.
enum : uint32_t {
  kInitPos = 0x10,
  kInitSpeed = 0x11,
  kInitMass = 0x12,
  kRelax = 0x20,
  kOrbit = 0x30,
  kSign = 0x31,
  kEnsemble = 0x40,
};

struct U4 {
  uint32_t x, y, z, w;
};

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): per round, two 32x32
// products of counter words 0 and 2 with fixed multipliers; the new words are
// (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key advances by two Weyl
// increments between rounds.
__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint64_t key) {
  uint32_t k0 = static_cast<uint32_t>(key), k1 = static_cast<uint32_t>(key >> 32);
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{c0, c1, c2, c3};
}

// Open-interval uniforms: (2x+1) 2^-53 from the top 52 bits of hi:lo, and
// (2x+1) 2^-24 from the top 23 bits of hi.  Both exact; they differ < 2^-23.
__device__ __forceinline__ double u01(uint32_t hi, uint32_t lo) {
  const uint64_t x = ((static_cast<uint64_t>(hi) << 32) | lo) >> 12;
  return static_cast<double>(2 * x + 1) * 0x1.0p-53;
}
__device__ __forceinline__ float u01f(uint32_t hi) {
  return static_cast<float>(2 * (hi >> 9) + 1) * 0x1.0p-24f;
}

// ---------------------------------------------------------------- LFSR113
// The generator of Sec. 3.6: L'Ecuyer's combined Tausworthe LFSR113.  Four
// component LFSRs of degrees k = 31, 29, 28, 25 with (q, s) = (6, 18),
// (2, 2), (13, 7), (3, 13); component c keeps the top k bits of its word and
// steps as b = ((z << q) ^ z) >> (k - s), z = ((z & top k bits) << s) ^ b;
// an output is the XOR of the four words.  A draw is one block of four
// consecutive outputs, in place of one Philox block.
struct alignas(16) Lfsr {
  uint32_t z[4];
};

template <int K, int Q, int S>
__device__ __forceinline__ uint32_t taus_step(uint32_t z) {
  const uint32_t b = ((z << Q) ^ z) >> (K - S);
  return ((z & (~0u << (32 - K))) << S) ^ b;
}

__device__ __forceinline__ uint32_t lfsr_next(Lfsr &g) {
  g.z[0] = taus_step<31, 6, 18>(g.z[0]);
  g.z[1] = taus_step<29, 2, 2>(g.z[1]);
  g.z[2] = taus_step<28, 13, 7>(g.z[2]);
  g.z[3] = taus_step<25, 3, 13>(g.z[3]);
  return g.z[0] ^ g.z[1] ^ g.z[2] ^ g.z[3];
}

__device__ __forceinline__ U4 lfsr_block(Lfsr &g) {
  U4 w;
  w.x = lfsr_next(g);
  w.y = lfsr_next(g);
  w.z = lfsr_next(g);
  w.w = lfsr_next(g);
  return w;
}

// A star's LFSR113 state in cmc_state.rng (4 words per star).
__device__ __forceinline__ Lfsr load_lfsr(const uint32_t *rng, int64_t k) {
  return reinterpret_cast<const Lfsr *>(rng)[k];
}
__device__ __forceinline__ void store_lfsr(uint32_t *rng, int64_t k, const Lfsr &g) {
  reinterpret_cast<Lfsr *>(rng)[k] = g;
}

// ---------------------------------------------------------------- reductions
// Deterministic: fixed butterfly inside a wave, fixed order across waves.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the block, valid in thread 0.  `sh` holds NT/64 entries.
template <int NT, typename T>
__device__ __forceinline__ T block_sum(T v, T *sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  T t = T(0);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) t += sh[i];
  }
  __syncthreads();
  return t;
}

// Inclusive prefix within the wave (lane order).
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T u = __shfl_up(v, o, 64);
    if (l >= o) v += u;
  }
  return v;
}

// Inclusive suffix within the wave (sum over lanes >= this lane).
template <typename T>
__device__ __forceinline__ T wave_incl_suffix(T v) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T u = __shfl_down(v, o, 64);
    if (l + o < 64) v += u;
  }
  return v;
}

// Exclusive prefix over the block (thread order); *total gets the block sum.
template <int NT, typename T>
__device__ __forceinline__ T block_excl_scan(T v, T *sh, T *total) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const T inc = wave_incl_scan(v);
  T exc = __shfl_up(inc, 1, 64);
  if (l == 0) exc = T(0);
  if (l == 63) sh[w] = inc;
  __syncthreads();
  T base = T(0), tot = T(0);
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) {
    if (i < w) base += sh[i];
    tot += sh[i];
  }
  __syncthreads();
  if (total) *total = tot;
  return base + exc;
}

// Exclusive suffix over the block: sum over threads with a larger index.
template <int NT, typename T>
__device__ __forceinline__ T block_excl_suffix(T v, T *sh, T *total) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const T inc = wave_incl_suffix(v);
  T exc = __shfl_down(inc, 1, 64);
  if (l == 63) exc = T(0);
  if (l == 0) sh[w] = inc;
  __syncthreads();
  T base = T(0), tot = T(0);
#pragma unroll
  for (int i = NT / 64 - 1; i >= 0; --i) {
    if (i > w) base += sh[i];
    tot += sh[i];
  }
  __syncthreads();
  if (total) *total = tot;
  return base + exc;
}

template <typename MT>
__device__ __forceinline__ double load_mass(const MT *m, int64_t k) {
  return static_cast<double>(m[k]);
}

__device__ __forceinline__ void set_status(cmc_scalars *sc, uint32_t bits) {
  if (bits) atomicOr(&sc->status, bits);
}

// ---------------------------------------------------------------- staging
// One star as it leaves the orbit pass (or the initial model) and waits for
// the sort.  The step's records carry the mass in the state's precision:
// with f32 masses a record is 32 bytes, one aligned quarter of a cache line,
// so the sort's random reads of records fetch one line each.  The initial
// model and cmc_sort stage f64 masses (WideRec).
template <typename MT>
struct StageRec;
template <>
struct alignas(32) StageRec<float> {
  double r, vr, vt;
  float m;
  uint32_t id;
};
template <>
struct alignas(8) StageRec<double> {
  double r, vr, vt, m;
  uint32_t id, pad;
};
using WideRec = StageRec<double>;
// An entry of the step's bucket sort: radius key, staged index, and the
// count of old radii <= r_new modulo the bucket span (see bucket.hip).
struct alignas(16) BktEnt {
  uint64_t key;
  uint32_t idx, sub;
};

// ---------------------------------------------------------------- orbit table
// The potential table as the orbit pass reads it.  Level 0 holds (r_k, Phi_k)
// for every star; level L >= 1 holds (r, Phi) of every 8^L-th star.  Each
// level starts 128-byte aligned, so the 8 children of a level-(L+1) sample
// are one aligned cache line of level L: a search descends one line per
// level (a static 8-ary B+tree in sampled-array form).  (M_k, S_k) sit in a
// parallel array read once per located interval.
struct alignas(16) RPhi {
  double r, phi;
};
struct alignas(16) MS {
  double M, S;
};
// Orbit of one star between the orbit pass's kernels, as two 32-byte halves:
// each turning point is found by one kernel, which writes its half whole
// (one aligned sector, no partial write).  lo: E, the lower turning point
// rmin in interval kmin (-1: inside the innermost star) and dQ/dr there;
// hi: J, rmax in interval kmax and dQ/dr there.  E >= 0 (or NaN) marks a
// star already sent out as an escaper.
struct alignas(32) OrbitLo {
  double E, rmin, dq;
  int32_t kmin;
  uint32_t pad;
};
struct alignas(32) OrbitHi {
  double J, rmax, dq;
  int32_t kmax;
  uint32_t pad;
};
struct alignas(64) OrbitRec {
  OrbitLo lo;
  OrbitHi hi;
};
// The grouped form writes each search's half where the search sits in the
// grouped order (32-byte slots over the orbit records' memory), and each
// star's two slots apart; a star that left has none.
constexpr uint32_t kNoPos = 0xFFFFFFFFu;
// One turning-point search left below the LDS-resident top levels: the
// star's E, J and index, and the sample of the level ltop the search reached
// (bit 31: the upper turning point).  Searches are grouped by that sample, so
// the ones that share a subtree of the table run together.
struct alignas(8) OrbQuery {
  double E, J;
  uint32_t i, node;
};
constexpr uint32_t kQueryHi = 0x80000000u;
constexpr int kMaxLevels = 12;  // 8^11 > 2^32 stars
struct Levels {
  RPhi *const *lev;  // the workspace's level pointers, [kMaxLevels]
  int nlev;          // levels in use for the capacity; the top one has <= 8 entries
};
// ---------------------------------------------------------------- radial index
// Buckets over the sorted radii.  The bucket of a radius x >= r_0 is
// (bits(x) - bits(r_0)) >> shift: the IEEE pattern of a non-negative double
// is monotone in its value and close to linear in log x, so buckets are
// roughly equal steps in log r.  start[b] is the first star whose bucket is
// >= b (start[nb] = n), so the stars with r_k <= x all lie below start[b+1]
// and all stars below start[b] have r_k < x.  shift makes the populated range
// fit nb = 2^lg_nb buckets.
struct RIndexCtl {
  uint64_t lo, hi;  // bits of r_0 and r_(n-1)
  uint32_t shift, n;
};
// Buckets [b0, b1) of the index that all take the value k.
struct alignas(16) RxRange {
  uint32_t b0, b1, k, pad;
};
constexpr int kRxShort = 32;     // bucket ranges one thread fills itself
constexpr int kRxPiece = 16384;  // longest range one block of the long-range pass fills
struct RIndex {
  const double *r;         // the sorted radii
  const uint32_t *start;   // [nb + 1]
  const RIndexCtl *ctl;
};

__device__ __forceinline__ uint64_t rbits(double x) { return __builtin_bit_cast(uint64_t, x + 0.0); }

// Last k with r_k <= x (-1 if none; n - 1 for x >= r_(n-1)).  c is *ix.ctl,
// loaded once by the caller.
__device__ __forceinline__ int64_t rindex_last_le(const RIndex &ix, const RIndexCtl &c,
                                                  double x) {
  const uint64_t kx = rbits(x);  // ordered like x for x >= 0
  if (kx < c.lo) return -1;
  if (kx >= c.hi) return static_cast<int64_t>(c.n) - 1;
  const uint64_t b = (kx - c.lo) >> c.shift;
  // (the bounds only matter for a table that was not sorted)
  int64_t lo = ix.start[b], hi = ix.start[b + 1];
  const int64_t n = static_cast<int64_t>(c.n);
  lo = lo < n ? lo : n;
  hi = hi < n ? hi : n;
  // r_k <= x for k < lo, r_k > x for k >= hi: the answer is the last k in
  // [lo - 1, hi - 1] with r_k <= x; halve long ranges, then scan
  while (hi - lo > 16) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (ix.r[mid] <= x) lo = mid + 1; else hi = mid;
  }
  for (;;) {
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = (lo + q < hi) ? ix.r[lo + q] : kInf;
    int c2 = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) c2 += (v[q] <= x) ? 1 : 0;
    lo += c2;
    if (c2 < 8 || lo >= hi) return lo - 1;
  }
}

// ---------------------------------------------------------------- workspace
constexpr int kSortTile = 4096;  // keys per radix tile (256 threads x 16)
constexpr int kPotTile = 1024;   // stars per potential tile (4 rounds of 256)
constexpr int kBlock = 256;
constexpr int kRedBlocks = 2048;  // grid of the grid-stride reduction kernels
constexpr int kKingNodes = 4096;  // nodes of a King profile: (r, W, M) each
// The step's sort (bucket.hip): bucket b holds the stars whose count of old
// radii <= r_new lies in [b * kBucketSpan, (b + 1) * kBucketSpan).
constexpr int kBucketShift = 11;
constexpr int64_t kBucketSpan = int64_t(1) << kBucketShift;  // old intervals per bucket
constexpr int kBucketBins = 16384;  // LDS bins of a tile: buckets of kept stars + escapers
constexpr int64_t kBucketCapMax = (kBucketBins - 1) * kBucketSpan - 1;  // largest capacity served
static_assert(kBucketCapMax == CMC_BUCKET_CAP_MAX, "the documented bucket-sort limit");
constexpr int kBucketTile = 16384;      // stars per histogram and scatter tile
constexpr int kBucketSortCap = 4096;    // stars a bucket sorts in LDS
constexpr uint32_t kBucketEsc = 0xFFFFFFFFu;  // bkey of a star that leaves the cluster
constexpr int kKingTab = 3 * kKingNodes + 8;
// The orbit table's top levels held in LDS by the orbit pass's kernels, and
// the sorted turning-point searches below them (orbit.hip).
// In LDS each 8-entry node of a level is followed by one unused entry: node
// s then starts on bank 36 s mod 64 of the 4-byte banks instead of all nodes
// on the same two, so the lanes of a wavefront that read the children of
// different nodes spread over the banks.
constexpr int kTopBytes = 52 * 1024;
constexpr int kTopEntries = kTopBytes / 16;  // LDS slots of 16 bytes, padding included
__host__ __device__ inline int64_t top_padded(int64_t len) { return len + (len >> 3) + 1; }
constexpr int kQueryTile = 4096;             // stars per tile of the search sort
constexpr int kQuerySearchBlock = 256;       // threads of the sorted-search kernel
constexpr int kQuerySearchChunk = 512;       // searches of one group per block of it
// Where a group's subtree spans at most kStagedLevels levels (8^4 = 4096
// stars), its search block holds the whole subtree in LDS, level 0 and the
// (M, S) of its stars included, and runs kStagedChunk searches of the group.
constexpr int kStagedLevels = 4;
constexpr int kStagedSpan = 1 << (3 * kStagedLevels);
constexpr int kStagedChunk = 16384;
constexpr int kStagedThreads = 1024;
constexpr int kStagedBlocks = 256;  // resident blocks of the staged search (one per CU)
constexpr int kPhiBins = 16384;  // bins of the potential-bound table (orbit.hip)
// LFSR113 stream seeding (rng.hip): for each component, the 32x32 bit matrix
// of 2^(80+b) steps for every bit b of a stream index (a base below 2^33
// plus a 32-bit star id), as 32 columns.
constexpr int kLfsrStreamBits = 34;
constexpr int kLfsrJumpWords = 4 * kLfsrStreamBits * 32;

struct Workspace {
  RPhi *lev[kMaxLevels];    // level L: [ceil(cap / 8^L)]
  int nlev;
  MS *ms;                   // [cap]
  OrbitRec *orec;           // [cap]
  void *stage;              // [cap] StageRec<MT> of the step, or WideRec
  uint64_t *keys[2];        // [cap]
  uint32_t *vals[2];        // [cap]
  uint32_t *tile_hist;      // [256 * sort_tiles]
  uint32_t *tile_off;       // [256 * sort_tiles]
  uint32_t *hist_all;       // [8 * 256]
  uint32_t *pass_info;      // [64]: skip mask, parity ...
  double *pot_tsum;         // [2 * pot_tiles]
  double *pot_carry;        // [2 * pot_tiles]
  double *pair_tp;          // [cap/2 + 1]
  double *pair_part;        // [4 * pair_blocks]
  double *dt_state;         // [32]
  double *red_part;         // [8 * star_blocks]  generic per-block partials
  uint32_t *rx_start;       // [rx_nb + 1] radial index buckets
  RxRange *rx_long;         // [rx_long_cap] bucket ranges too long for one thread
  uint32_t *rx_nlong;       // [1] ranges in rx_long
  RIndexCtl *rx_ctl;        // [1]
  double *king;             // [kKingTab] King model profile (initial model only)
  double *phib;             // [kPhiBins + 1] Phi at the bound table's edge radii
  uint64_t *phib_ctl;       // [2]: bits of the first edge, shift from bits to bins
  uint32_t *bkey;           // [cap] old radii <= each staged radius, or kBucketEsc
  BktEnt *bent;             // [cap] entries grouped by bucket (shares orec's memory)
  uint32_t *bkt_cnt;        // [bkt_tiles * bkt_bins] per-tile counts, then tile offsets
  uint32_t *bkt_tot;        // [bkt_bins] stars per bucket
  uint32_t *bkt_start;      // [bkt_bins + 1] first position of each bucket
  int64_t *bkt_info;        // [2]: staged stars, kept stars
  RPhi *cor;                // [cap] energy correction, old order: (r_old, Phi_old(r_old))
  double *pn;               // [cap] Phi_old(r_new), then the summed work terms
  uint32_t *perm;           // [cap] staged (old) index of each sorted star
  Lfsr *rng_stage;          // [cap] LFSR113 states after the orbit pass, staged order
  uint32_t *lfsr_jump;      // [kLfsrJumpWords] jump matrices of the stream seeding
  OrbQuery *oq;             // [2 cap] turning-point searches grouped by top sample
  uint32_t *oq_cnt;         // [oq_tiles * oq_bins] per-tile counts, then tile offsets
  uint32_t *oq_tot;         // [oq_bins] searches per top sample
  uint32_t *oq_start;       // [oq_bins + 1] first search of each top sample
  uint32_t *oq_chunk;       // [oq_bins + 1] first search block of each top sample,
                            // then the staged search's work counter
  uint32_t *oq_bmap;        // [search blocks] the top sample each search block works on
  uint32_t *oq_node;        // [cap] each star's two top samples
  uint32_t *oq_pos;         // [2 cap] each star's two halves in the grouped form's
                            // results (kNoPos: none, the star left)
  int64_t bkt_bins, bkt_tiles;  // bkt_bins = 0: capacity above kBucketCapMax
  int64_t oq_bins, oq_tiles;    // groups (samples of the level the LDS top ends at,
                                // and one more); tiles
  int32_t oq_staged;            // the groups' searches run with the subtree in LDS
  // launch settings from the launch table (cluster_args; layout() leaves the
  // built-in defaults)
  int32_t sorted, bracket_blocks, trial_chunk;
  int64_t rx_nb;
  int64_t rx_long_cap;
  int rx_lg_nb;
  int64_t sort_tiles, pot_tiles, pair_blocks, star_blocks;
  size_t bytes;
};

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Top levels of the orbit table kept in LDS: levels from the top down while
// they fit kTopBytes (at the capacity).  ltop = the lowest of them.
struct OrbitTop {             // top levels of the orbit table kept in LDS
  int32_t off[kMaxLevels];    // LDS slot of level L's entry 0, for L >= ltop (entry
                              // e of the level at slot off + e + e / 8)
  int32_t len[kMaxLevels];    // entries of level L at the capacity
  int32_t ltop, entries;
};
inline OrbitTop top_levels(int nlev, int64_t cap) {
  OrbitTop tl{};
  int64_t tot = 0;
  tl.ltop = nlev;
  for (int L = nlev - 1; L >= 0; --L) {
    const int64_t stride = int64_t(1) << (3 * L);
    const int64_t len = (cap + stride - 1) / stride;
    if ((tot + top_padded(len)) * 16 > kTopBytes) break;
    tl.off[L] = static_cast<int32_t>(tot);
    tl.len[L] = static_cast<int32_t>(len);
    tot += top_padded(len);
    tl.ltop = L;
  }
  tl.entries = static_cast<int32_t>(tot);
  return tl;
}

constexpr int kDefaultBracketBlocks = 1024;  // resident bracket blocks of one cluster
constexpr int kDefaultTrialChunk = 128;      // stars per wavefront chunk of the trial kernel
constexpr int kMaxTrialChunk = 1024;         // the launch table's largest chunk

inline Workspace layout(int64_t cap, void *base) {
  Workspace w{};
  char *p = static_cast<char *>(base);
  size_t off = 0;
  auto take = [&](size_t bytes) -> char * {
    off = (off + 255) & ~size_t(255);
    char *q = p ? p + off : nullptr;
    off += bytes;
    return q;
  };
  const int64_t c = cap > 0 ? cap : 1;
  w.sort_tiles = cdiv(c, kSortTile);
  w.pot_tiles = cdiv(c, kPotTile);
  w.pair_blocks = cdiv(c / 2 + 1, kBlock);
  w.star_blocks = cdiv(c, kBlock);
  {
    int64_t len = c;
    w.nlev = 0;
    for (;;) {
      w.lev[w.nlev++] = reinterpret_cast<RPhi *>(take(sizeof(RPhi) * len));
      if (len <= 8 || w.nlev == kMaxLevels) break;
      len = (len + 7) / 8;
    }
    for (int L = w.nlev; L < kMaxLevels; ++L) w.lev[L] = nullptr;
  }
  w.ms = reinterpret_cast<MS *>(take(sizeof(MS) * c));
  w.orec = reinterpret_cast<OrbitRec *>(take(sizeof(OrbitRec) * c));
  w.stage = take(sizeof(WideRec) * c);
  static_assert(sizeof(WideRec) >= sizeof(StageRec<float>), "stage holds either record");
  w.keys[0] = reinterpret_cast<uint64_t *>(take(8 * c));
  w.keys[1] = reinterpret_cast<uint64_t *>(take(8 * c));
  w.vals[0] = reinterpret_cast<uint32_t *>(take(4 * c));
  w.vals[1] = reinterpret_cast<uint32_t *>(take(4 * c));
  w.tile_hist = reinterpret_cast<uint32_t *>(take(4 * 256 * w.sort_tiles));
  w.tile_off = reinterpret_cast<uint32_t *>(take(4 * 256 * w.sort_tiles));
  w.hist_all = reinterpret_cast<uint32_t *>(take(4 * 8 * 256));
  w.pass_info = reinterpret_cast<uint32_t *>(take(4 * 64));
  w.pot_tsum = reinterpret_cast<double *>(take(8 * 2 * w.pot_tiles));
  w.pot_carry = reinterpret_cast<double *>(take(8 * 2 * w.pot_tiles));
  w.pair_tp = reinterpret_cast<double *>(take(8 * (c / 2 + 1)));
  w.pair_part = reinterpret_cast<double *>(take(8 * 4 * w.pair_blocks));
  w.dt_state = reinterpret_cast<double *>(take(8 * 32));
  w.red_part = reinterpret_cast<double *>(take(8 * 8 * w.star_blocks));
  // at least one bucket per star: a trial radius's scan then stays within a
  // line of the radii where stars crowd; halving the buckets makes the
  // trials slower by more than the smaller index saves in building it
  w.rx_lg_nb = 0;
  while ((int64_t(1) << w.rx_lg_nb) < c + 1) ++w.rx_lg_nb;
  w.rx_nb = int64_t(1) << w.rx_lg_nb;
  w.rx_start = reinterpret_cast<uint32_t *>(take(4 * (w.rx_nb + 1)));
  // ranges longer than kRxShort are disjoint, and none is longer than
  // kRxPiece after the split: at most this many pieces
  w.rx_long_cap = cdiv(w.rx_nb + 1, kRxShort + 1) + cdiv(w.rx_nb + 1, kRxPiece) + 1;
  w.rx_long = reinterpret_cast<RxRange *>(take(sizeof(RxRange) * w.rx_long_cap));
  w.rx_nlong = reinterpret_cast<uint32_t *>(take(4));
  w.rx_ctl = reinterpret_cast<RIndexCtl *>(take(sizeof(RIndexCtl)));
  w.king = reinterpret_cast<double *>(take(8 * kKingTab));
  w.phib = reinterpret_cast<double *>(take(8 * (kPhiBins + 1)));
  w.phib_ctl = reinterpret_cast<uint64_t *>(take(8 * 2));
  w.bkey = reinterpret_cast<uint32_t *>(take(4 * c));
  w.cor = reinterpret_cast<RPhi *>(take(sizeof(RPhi) * c));
  w.pn = reinterpret_cast<double *>(take(8 * c));
  w.perm = reinterpret_cast<uint32_t *>(take(4 * c));
  w.rng_stage = reinterpret_cast<Lfsr *>(take(sizeof(Lfsr) * c));
  w.lfsr_jump = reinterpret_cast<uint32_t *>(take(4 * kLfsrJumpWords));
  {
    const OrbitTop tl = top_levels(w.nlev, c);
    // the groups: one per sample of level ltop, and one for the lower turning
    // points the LDS levels already finish
    w.oq_bins = tl.ltop > 0 ? tl.len[tl.ltop] + 1 : 1;
    w.oq_staged = (tl.ltop > 0 && tl.ltop <= kStagedLevels) ? 1 : 0;
    w.oq_tiles = cdiv(c, kQueryTile);
    w.oq = reinterpret_cast<OrbQuery *>(take(sizeof(OrbQuery) * 2 * c));
    w.oq_cnt = reinterpret_cast<uint32_t *>(take(4 * w.oq_tiles * w.oq_bins));
    w.oq_tot = reinterpret_cast<uint32_t *>(take(4 * w.oq_bins));
    w.oq_start = reinterpret_cast<uint32_t *>(take(4 * (w.oq_bins + 1)));
    // (+ the staged search's work counter at oq_bins + 1)
    w.oq_chunk = reinterpret_cast<uint32_t *>(take(4 * (w.oq_bins + 2)));
    w.oq_bmap = reinterpret_cast<uint32_t *>(take(4 * (w.oq_bins + cdiv(2 * c, kQuerySearchChunk))));
    w.oq_node = reinterpret_cast<uint32_t *>(take(4 * c));
    w.oq_pos = reinterpret_cast<uint32_t *>(take(8 * c));
  }
  w.bent = reinterpret_cast<BktEnt *>(w.orec);  // orec is dead once the orbit pass ends
  static_assert(sizeof(BktEnt) <= sizeof(OrbitRec), "bent fits in orec");
  if (c <= kBucketCapMax) {
    w.bkt_bins = (c >> kBucketShift) + 2;
    w.bkt_tiles = cdiv(c, kBucketTile);
    w.bkt_cnt = reinterpret_cast<uint32_t *>(take(4 * w.bkt_tiles * w.bkt_bins));
    w.bkt_tot = reinterpret_cast<uint32_t *>(take(4 * w.bkt_bins));
    w.bkt_start = reinterpret_cast<uint32_t *>(take(4 * (w.bkt_bins + 1)));
    w.bkt_info = reinterpret_cast<int64_t *>(take(8 * 2));
  }
  w.sorted = 0;
  w.bracket_blocks = kDefaultBracketBlocks;
  w.trial_chunk = kDefaultTrialChunk;
  w.bytes = (off + 255) & ~size_t(255);
  return w;
}

// A view of the workspace's levels (no copy: kernels index it with
// run-time level numbers).
__host__ __device__ inline Levels levels_of(const Workspace &w) { return Levels{w.lev, w.nlev}; }

// Write star k's table entries (level 0, every level L whose stride divides
// k, and M, S).
__device__ __forceinline__ void put_table(const Levels &lv, MS *ms, int64_t k, double r,
                                          double phi, double M, double S) {
  const RPhi e{r, phi};
  lv.lev[0][k] = e;
  ms[k] = MS{M, S};
  int64_t q = k;
  for (int L = 1; L < lv.nlev && (q & 7) == 0; ++L) {
    q >>= 3;
    lv.lev[L][q] = e;
  }
}

// ---------------------------------------------------------------- column scan
// The counting sorts' tile offsets.  cnt is a table of counts, row t for
// tile t (rows stride apart); for the G columns c0 .. c0 + G - 1 below ncol,
// every entry becomes the sum of its column above it (the tile's offset
// inside the column) and tot[c] the column's total.  A block of NTB
// threads: thread x takes column x mod G and one of NTB / G contiguous runs
// of tiles, so a wave reads 64 / G runs of G adjacent counts and the grid has
// one block per G columns.
constexpr int kQColGroup = 16;    // the search sort: few tiles, few groups
constexpr int kBktColGroup = 64;  // the step's sort
template <int NTB, int G>
__device__ __forceinline__ void column_scan(uint32_t *__restrict__ cnt, int64_t stride,
                                            int64_t tiles, int64_t c0, int64_t ncol,
                                            uint32_t *__restrict__ tot) {
  constexpr int R = NTB / G;
  __shared__ uint32_t part[R][G];
  const int col = static_cast<int>(threadIdx.x) % G;
  const int run = static_cast<int>(threadIdx.x) / G;
  const int64_t c = c0 + col;
  const bool own = c < ncol;
  const int64_t per = cdiv(tiles, int64_t(R));
  const int64_t t0 = run * per;
  const int64_t t1 = t0 + per < tiles ? t0 + per : tiles;
  // (each thread's run is read kScanBatch entries at a time, all in flight:
  // the run is a chain of dependent steps otherwise)
  constexpr int kScanBatch = 8;
  uint32_t s = 0u;
  if (own) {
    for (int64_t t = t0; t < t1; t += kScanBatch) {
      uint32_t v[kScanBatch];
#pragma unroll
      for (int u = 0; u < kScanBatch; ++u) v[u] = t + u < t1 ? cnt[(t + u) * stride + c] : 0u;
#pragma unroll
      for (int u = 0; u < kScanBatch; ++u) s += v[u];
    }
  }
  part[run][col] = s;
  __syncthreads();
  uint32_t pre = 0u, all = 0u;
  for (int q = 0; q < R; ++q) {
    const uint32_t v = part[q][col];
    if (q < run) pre += v;
    all += v;
  }
  if (!own) return;
  if (run == 0) tot[c] = all;
  for (int64_t t = t0; t < t1; t += kScanBatch) {
    uint32_t v[kScanBatch];
#pragma unroll
    for (int u = 0; u < kScanBatch; ++u) v[u] = t + u < t1 ? cnt[(t + u) * stride + c] : 0u;
#pragma unroll
    for (int u = 0; u < kScanBatch; ++u) {
      if (t + u < t1) cnt[(t + u) * stride + c] = pre;
      pre += v[u];
    }
  }
}

// ---------------------------------------------------------------- launch context
// What a kernel knows about the cluster it works on.  One cluster: the
// arguments travel by value and block b of the launch is block b of the
// cluster.  An ensemble: one launch covers every cluster, each cluster owns
// its own arrays and workspace, and a per-shape map names the cluster of
// each block and the cluster's first block.
struct ClusterArgs {
  cmc_state s;                // the cluster's arrays (device pointers)
  Workspace w;                // its workspace
  OrbitTop top;
  uint64_t seed;              // Philox key
  double gamma;               // Coulomb logarithm ln(gamma N)
  int32_t model;              // initial model: CMC_MODEL_PLUMMER or CMC_MODEL_KING
  int32_t mass_spectrum;      // 1: broken power-law masses
  double w0;                  // King central potential W0
  int64_t n_init;             // stars the initial model draws
  int64_t bracket_blocks;     // blocks of the cluster in the bracket kernel
};

struct One {
  ClusterArgs a;
  __device__ __forceinline__ int index() const { return 0; }
  __device__ __forceinline__ const ClusterArgs &args() const { return a; }
  __device__ __forceinline__ int64_t block() const { return blockIdx.x; }
  __device__ __forceinline__ int64_t nblocks() const { return gridDim.x; }
};
struct Many {
  const ClusterArgs *a;       // [clusters]
  const uint16_t *map;        // [blocks of the launch]: the block's cluster
  const int64_t *first;       // [clusters + 1]: first block of each cluster
  __device__ __forceinline__ int c() const { return map[blockIdx.x]; }
  __device__ __forceinline__ int index() const { return c(); }
  __device__ __forceinline__ const ClusterArgs &args() const { return a[c()]; }
  __device__ __forceinline__ int64_t block() const { return blockIdx.x - first[c()]; }
  __device__ __forceinline__ int64_t nblocks() const {
    const int cc = c();
    return first[cc + 1] - first[cc];
  }
};

// The step index of a call: its own, or the cluster's device counter for
// calls replayed from a captured graph.
__device__ __forceinline__ uint32_t step_of(const ClusterArgs &A, uint32_t step) {
  return step == CMC_STEP_DEVICE ? static_cast<uint32_t>(A.s.sc->step) : step;
}

// Launch shapes: blocks per cluster of each kind of grid.
enum Shape : int {
  kShOne,       // one block per cluster
  kShStar,      // one thread per star, 256 per block
  kShPair,      // one thread per pair
  kShDtEval,    // grid-stride over pairs, at most kRedBlocks blocks
  kShPotTile,   // potential tiles
  kShSortTile,  // radix tiles
  kShKeyRange,  // grid-stride over keys, at most 1024 blocks
  kShDigit,     // one block per radix digit
  kShBracket,   // resident blocks of the bracket kernel
  kShTrials,    // wavefront chunks of the trial kernel
  kShRxFill,    // one thread per star (at least one), fills the bucket index
  kShRxLong,    // grid-stride over the bucket index's long ranges
  kShDiag,      // grid-stride diagnostics partials
  kShBktTile,   // histogram and scatter tiles of the step's sort
  kShBktGroup,  // groups of kBktColGroup buckets
  kShBktSort,   // one block per bucket of kept stars
  kShQTile,     // tiles of the orbit pass's search sort
  kShQGroup,    // groups of kQColGroup top samples
  kShQSearch,   // blocks of sorted turning-point searches (subtree below the LDS)
  kShQStaged,   // resident blocks of sorted turning-point searches (subtree in LDS)
  kShapes
};
constexpr int kBracketThreads = 512;
__host__ __device__ inline int64_t blocks_of(Shape sh, const Workspace &w, int64_t cap) {
  const int64_t c = cap > 0 ? cap : 1;
  switch (sh) {
    case kShOne: return 1;
    case kShStar: return w.star_blocks;
    case kShPair: return w.pair_blocks;
    case kShDtEval: return w.pair_blocks < kRedBlocks ? w.pair_blocks : kRedBlocks;
    case kShPotTile: return w.pot_tiles;
    case kShSortTile: return w.sort_tiles;
    case kShKeyRange: return w.sort_tiles < 1024 ? w.sort_tiles : 1024;
    case kShDigit: return 256;
    case kShBracket: {
      const int64_t b = cdiv(c, kBracketThreads);
      return b < w.bracket_blocks ? b : w.bracket_blocks;
    }
    case kShTrials: return cdiv(c, int64_t(w.trial_chunk) * (kBlock / 64));
    case kShRxFill: return w.star_blocks;
    case kShRxLong: {
      const int64_t b = cdiv(w.rx_nb + 1, kRxPiece);
      return b < 1024 ? b : 1024;
    }
    case kShDiag: return w.star_blocks < kRedBlocks ? w.star_blocks : kRedBlocks;
    case kShBktTile: return w.bkt_bins ? w.bkt_tiles : 1;
    case kShBktGroup: return w.bkt_bins ? cdiv(w.bkt_bins, int64_t(kBktColGroup)) : 1;
    case kShBktSort: return w.bkt_bins ? w.bkt_bins - 1 : 1;
    case kShQTile: return w.oq_tiles;
    case kShQGroup: return cdiv(w.oq_bins, int64_t(kQColGroup));
    // one form or the other, by the subtree's depth
    case kShQSearch: return w.oq_staged ? 0 : w.oq_bins + cdiv(2 * c, kQuerySearchChunk);
    case kShQStaged: {
      const int64_t b = w.oq_bins + cdiv(2 * c, kStagedChunk);
      return w.oq_staged ? (b < kStagedBlocks ? b : kStagedBlocks) : 0;
    }
    default: return 1;
  }
}

// Host side of a launch: one cluster, or an ensemble whose tables live in
// device memory (see batch.hip).
struct BatchDev {
  int32_t clusters;
  const ClusterArgs *args;              // device [clusters]
  const uint16_t *map[kShapes];         // device, per shape
  const int64_t *first[kShapes];        // device, per shape [clusters + 1]
  int64_t total[kShapes];               // blocks per shape over all clusters
  int32_t top_entries;                  // largest OrbitTop::entries
  int32_t any_f32, any_f64;             // mass storage kinds present
  int32_t bucket_sort;                  // every cluster's capacity <= kBucketCapMax
  int32_t sorted;                       // the orbit pass groups its searches
};
struct Target {
  const ClusterArgs *one;               // host struct, or null
  const BatchDev *many;                 // or an ensemble
};
struct OneL {
  const ClusterArgs &a;
  One ctx(Shape) const { return One{a}; }
  unsigned grid(Shape sh) const { return static_cast<unsigned>(blocks_of(sh, a.w, a.s.cap)); }
  int top_entries() const { return a.top.entries; }
  // whether some cluster's table fits the LDS whole (its star pass then
  // searches with the LDS levels alone)
  bool flat_top() const { return a.top.ltop == 0; }
};
struct ManyL {
  const BatchDev &d;
  Many ctx(Shape sh) const { return Many{d.args, d.map[sh], d.first[sh]}; }
  unsigned grid(Shape sh) const { return static_cast<unsigned>(d.total[sh]); }
  int top_entries() const { return d.top_entries; }
  bool flat_top() const { return true; }
};

// The orbit table's LDS-resident top levels for a capacity.
OrbitTop orbit_top(const Workspace &w, int64_t cap);
ClusterArgs cluster_args(const cmc_state &s, uint64_t seed, double gamma);


// ---------------------------------------------------------------- launchers
// Defined in the translation units; each returns hipGetLastError().  Masses
// are f32 or f64 per cluster; an ensemble must not mix the two.
// public_arrays: also write phi, mcum, ssuf of the state (the orbit pass
// reads only the workspace table)
hipError_t launch_potential(const Target &t, bool m_f32, int precision, bool public_arrays,
                            hipStream_t st);
// phi, mcum, ssuf of the state without the orbit table: the workspace need
// only hold pot_tsum and pot_carry (pot_tiles of them).
hipError_t launch_potential_public_only(const Target &t, bool m_f32, int precision,
                                        hipStream_t st);
hipError_t launch_timestep(const Target &t, bool m_f32, const cmc_params &p, hipStream_t st);
hipError_t launch_relax(const Target &t, bool m_f32, const cmc_params &p, hipStream_t st);
// corr: also record each star's energy-correction terms (cor, pn);
// rindex_ready: the radial index of the sorted radii is already built.
hipError_t launch_orbit(const Target &t, bool m_f32, const cmc_params &p, bool to_stage,
                        bool corr, bool rindex_ready, hipStream_t st);
hipError_t launch_table_pack(const Target &t, hipStream_t st);
hipError_t launch_rindex(const Target &t, hipStream_t st);
hipError_t launch_stage_from_state(const Target &t, bool m_f32, hipStream_t st);
// Radix sort of the staged records by keys[0]: the step's records
// (StageRec<mass type>) or WideRec.  corr: write perm and leave the energy
// correction pending (sc->corr_n = staged stars); else clear it.
hipError_t launch_sort_stage(const Target &t, bool m_f32, bool normalise_mass, bool step_records,
                             bool corr, bool move_rng, hipStream_t st);
hipError_t launch_init(const Target &t, bool m_f32, hipStream_t st);
hipError_t launch_diagnostics(const Target &t, bool m_f32, double *out, hipStream_t st);
hipError_t launch_philox(uint64_t key, const uint32_t *ctr, uint32_t *out, int64_t n,
                         hipStream_t st);
// LFSR113 (rng.hip): every star's stream state, and raw words.
hipError_t launch_lfsr_seed(const Target &t, const uint32_t z0[4], uint64_t stream_base,
                            hipStream_t st);
hipError_t launch_lfsr_words(const uint32_t *state, uint32_t *out, int64_t n, int32_t blocks,
                             hipStream_t st);
hipError_t launch_step(const Target &t, bool m_f32, const cmc_params &p, void *const *events,
                       hipStream_t st);
hipError_t launch_step_advance(const Target &t, hipStream_t st);
// The step's sort of the orbit pass's staged records (stage, bkey) into the
// state; capacities above kBucketCapMax take the radix sort instead.
hipError_t launch_bucket_sort(const Target &t, bool m_f32, bool corr, hipStream_t st);
// The pending energy correction (energy.hip), after the potential of the
// state the step left: builds the radial index, applies it, and with
// `finish` clears sc->corr_n.
hipError_t launch_energy_correction(const Target &t, bool finish, hipStream_t st);
// Whether the orbit pass groups its turning-point searches (orbit.hip), as
// the launch table chose for the cluster or the ensemble.
inline bool sorted_searches(const Target &t) {
  if (t.many) return t.many->sorted != 0;
  return t.one->w.sorted != 0;
}
// The launch table (capi.hip): the entry serving a capacity, and its
// settings into a workspace view.
cmc_tuning tuning_for(int64_t cap);
void apply_tuning(Workspace &w, const cmc_tuning &t);
// Whether the target's step sorts by buckets.
inline bool bucket_sort_of(const Target &t) {
  return t.many ? t.many->bucket_sort != 0 : t.one->w.bkt_bins > 0;
}

// Run F<One or Many launch> on the target.
template <class F>
hipError_t dispatch(const Target &t, F &&f) {
  if (t.many) return f(ManyL{*t.many});
  return f(OneL{*t.one});
}

}  // namespace cmc

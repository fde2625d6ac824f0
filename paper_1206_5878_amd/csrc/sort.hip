// sort.hip -- radial sort (arXiv:1206.5878, Sec. 2.1 step 6), replacing the
// paper's Quicksort / sample sort by a stable LSD radix sort on gfx950.
//
// Key of a star: the bit pattern of r_new + 0.0 as an unsigned integer, which
// orders non-negative radii (and +inf) numerically.  Keys are compressed to
// key - min_key over the finite keys, non-finite keys (escapers) map to
// range + 1, so only ceil(bits(range + 1) / 8) digit passes run.  Each pass:
// per-tile digit histograms in LDS, a per-digit scan over tiles, and a
// scatter in which every wavefront ranks its keys with 8 ballots per slot
// (stable: tile order = wave, slot, lane = input order).  Values are the
// star's index in the staged records; a final gather writes the SoA arrays.
#include <algorithm>

#include "cmc_internal.hpp"

namespace cmc {
namespace {

constexpr int NT = kBlock;           // 4 waves
constexpr int SLOTS = kSortTile / NT;  // 16 keys per thread
constexpr int DT = 512;                 // threads of the downsweep
constexpr int DSLOTS = kSortTile / DT;  // its keys per thread
constexpr uint64_t kInfKey = 0x7FF0000000000000ull;

// pass_info as uint64 slots
enum { kNTotal = 0, kNKept, kPasses, kMinKey, kMaxKey, kNonFin, kEscKey };

__device__ __forceinline__ uint64_t radius_key(double x) {
  return __builtin_bit_cast(uint64_t, x + 0.0);
}

// One thread per cluster.
template <class Ctx>
__global__ void k_sort_prep(Ctx ctx) {
  const ClusterArgs &A = ctx.args();
  uint64_t *__restrict__ pi = reinterpret_cast<uint64_t *>(A.w.pass_info);
  pi[kNTotal] = static_cast<uint64_t>(A.s.sc->n);
  pi[kMinKey] = ~0ull;
  pi[kMaxKey] = 0ull;
  pi[kNonFin] = 0ull;
}

template <class Ctx>
__global__ __launch_bounds__(NT) void k_stage_from_state(Ctx ctx) {
  const ClusterArgs &A = ctx.args();
  const int64_t n = A.s.sc->n;
  const int64_t i = ctx.block() * NT + threadIdx.x;
  if (i >= n) return;
  WideRec rec;
  rec.r = A.s.r_new[i];
  rec.vr = A.s.vr[i];
  rec.vt = A.s.vt[i];
  rec.m = A.s.m_f32 ? static_cast<double>(static_cast<const float *>(A.s.m)[i])
                    : static_cast<const double *>(A.s.m)[i];
  rec.id = A.s.id[i];
  rec.pad = 0u;
  static_cast<WideRec *>(A.w.stage)[i] = rec;
  A.w.keys[0][i] = radius_key(rec.r);
  if (A.s.rng) A.w.rng_stage[i] = load_lfsr(A.s.rng, i);  // moves with its star
}

// Per-block min and max of the finite keys and count of non-finite ones;
// k_plan combines the blocks' partials (no contended atomics).
template <class Ctx>
__global__ __launch_bounds__(NT) void k_key_range(Ctx ctx) {
  __shared__ uint64_t smin[NT / 64], smax[NT / 64];
  __shared__ uint32_t snf[NT / 64];
  const ClusterArgs &A = ctx.args();
  const uint64_t *__restrict__ keys = A.w.keys[0];
  const uint64_t *__restrict__ pi = reinterpret_cast<const uint64_t *>(A.w.pass_info);
  uint64_t *__restrict__ part = reinterpret_cast<uint64_t *>(A.w.red_part);
  const int64_t n = static_cast<int64_t>(pi[kNTotal]);
  const int64_t blk = ctx.block();
  uint64_t lo = ~0ull, hi = 0ull;
  uint32_t nf = 0;
  for (int64_t k = blk * NT + threadIdx.x; k < n; k += ctx.nblocks() * NT) {
    const uint64_t x = keys[k];
    if (x < kInfKey) {
      lo = x < lo ? x : lo;
      hi = x > hi ? x : hi;
    } else {
      ++nf;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t a = __shfl_xor(lo, o, 64), b = __shfl_xor(hi, o, 64);
    lo = a < lo ? a : lo;
    hi = b > hi ? b : hi;
    nf += __shfl_xor(nf, o, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    smin[w] = lo;
    smax[w] = hi;
    snf[w] = nf;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < NT / 64; ++q) {
      lo = smin[q] < lo ? smin[q] : lo;
      hi = smax[q] > hi ? smax[q] : hi;
      nf += snf[q];
    }
    part[3 * blk] = lo;
    part[3 * blk + 1] = hi;
    part[3 * blk + 2] = nf;
  }
}

// One block per cluster.  Also leaves the staged stars' energy correction
// pending (corr) or none.
template <class Ctx>
__global__ __launch_bounds__(NT) void k_plan(Ctx ctx, int corr) {
  __shared__ uint64_t smin[NT / 64], smax[NT / 64], snf[NT / 64];
  const ClusterArgs &A = ctx.args();
  const uint64_t *__restrict__ part = reinterpret_cast<const uint64_t *>(A.w.red_part);
  const int64_t nparts = blocks_of(kShKeyRange, A.w, A.s.cap);
  uint64_t *__restrict__ pi = reinterpret_cast<uint64_t *>(A.w.pass_info);
  cmc_scalars *__restrict__ sc = A.s.sc;
  uint64_t lo = ~0ull, hi = 0ull, nfin = 0ull;
  for (int64_t b = threadIdx.x; b < nparts; b += NT) {
    lo = part[3 * b] < lo ? part[3 * b] : lo;
    hi = part[3 * b + 1] > hi ? part[3 * b + 1] : hi;
    nfin += part[3 * b + 2];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t a = __shfl_xor(lo, o, 64), b = __shfl_xor(hi, o, 64);
    lo = a < lo ? a : lo;
    hi = b > hi ? b : hi;
    nfin += __shfl_xor(nfin, o, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    smin[w] = lo;
    smax[w] = hi;
    snf[w] = nfin;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int q = 1; q < NT / 64; ++q) {
    lo = smin[q] < lo ? smin[q] : lo;
    hi = smax[q] > hi ? smax[q] : hi;
    nfin += snf[q];
  }
  const uint64_t n = pi[kNTotal], nf = nfin;
  const uint64_t kept = n - nf;
  const uint64_t range = kept ? hi - lo : 0ull;
  const uint64_t esc = range + 1ull;
  const uint64_t top = nf ? esc : range;
  int bits = 0;
  while (bits < 64 && (top >> bits) != 0ull) ++bits;
  pi[kPasses] = (n <= 1) ? 0ull : static_cast<uint64_t>((bits + 7) / 8);
  pi[kNKept] = kept;
  pi[kEscKey] = esc;
  pi[kMinKey] = kept ? lo : 0ull;
  pi[kMaxKey] = hi;
  pi[kNonFin] = nf;
  sc->n = static_cast<int64_t>(kept);
  sc->corr_n = corr ? static_cast<int64_t>(n) : 0;
}

// key of item k for pass 0 (compression applied) or a later pass
__device__ __forceinline__ uint64_t pass_key(const uint64_t *__restrict__ in, int64_t k,
                                             bool first, uint64_t kmin, uint64_t esc) {
  const uint64_t x = in[k];
  if (!first) return x;
  return x < kInfKey ? x - kmin : esc;
}

template <class Ctx>
__global__ __launch_bounds__(NT) void k_upsweep(Ctx ctx, int pass) {
  __shared__ uint32_t hist[256];
  const ClusterArgs &A = ctx.args();
  const uint64_t *keys0 = A.w.keys[0];
  const uint64_t *keys1 = A.w.keys[1];
  const uint64_t *__restrict__ pi = reinterpret_cast<const uint64_t *>(A.w.pass_info);
  uint32_t *__restrict__ tile_hist = A.w.tile_hist;
  const int64_t tiles = A.w.sort_tiles;
  const int64_t blk = ctx.block();
  if (static_cast<uint64_t>(pass) >= pi[kPasses]) return;
  const int64_t n = static_cast<int64_t>(pi[kNTotal]);
  const uint64_t *in = (pass & 1) ? keys1 : keys0;
  const uint64_t kmin = pi[kMinKey], esc = pi[kEscKey];
  const int shift = 8 * pass;
  hist[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t base = blk * kSortTile;
  for (int j = 0; j < SLOTS; ++j) {
    const int64_t k = base + j * NT + threadIdx.x;
    if (k < n) {
      const uint32_t d = static_cast<uint32_t>(pass_key(in, k, pass == 0, kmin, esc) >> shift) & 255u;
      atomicAdd(&hist[d], 1u);
    }
  }
  __syncthreads();
  tile_hist[static_cast<int64_t>(threadIdx.x) * tiles + blk] = hist[threadIdx.x];
}

// Block d: exclusive scan of digit d's counts over tiles; total in digit_tot[d].
template <class Ctx>
__global__ __launch_bounds__(NT) void k_scan_digits(Ctx ctx, int pass) {
  __shared__ uint32_t sh[NT / 64];
  const ClusterArgs &A = ctx.args();
  const uint32_t *__restrict__ tile_hist = A.w.tile_hist;
  const uint64_t *__restrict__ pi = reinterpret_cast<const uint64_t *>(A.w.pass_info);
  uint32_t *__restrict__ tile_off = A.w.tile_off;
  uint32_t *__restrict__ digit_tot = A.w.hist_all;
  const int64_t tiles = A.w.sort_tiles;
  if (static_cast<uint64_t>(pass) >= pi[kPasses]) return;
  const int64_t d = ctx.block();
  const uint32_t *h = tile_hist + d * tiles;
  uint32_t *o = tile_off + d * tiles;
  uint32_t carry = 0u;
  for (int64_t t0 = 0; t0 < tiles; t0 += NT) {
    const int64_t t = t0 + threadIdx.x;
    const uint32_t v = t < tiles ? h[t] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan<NT>(v, sh, &tot);
    if (t < tiles) o[t] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) digit_tot[d] = carry;
}

// The in and out buffers of a pass are the two halves of one ping-pong pair,
// so they carry no restrict qualifier.  Keys are ranked in registers, placed
// in digit order in LDS, then written out in LDS order, so consecutive
// lanes write consecutive addresses of one digit's run.
template <class Ctx>
__global__ __launch_bounds__(DT) void k_downsweep(Ctx ctx, int pass) {
  __shared__ uint32_t cnt[DT / 64][256];
  __shared__ uint32_t gdelta[256];
  __shared__ uint32_t sh[DT / 64];
  __shared__ uint64_t lkey[kSortTile];
  __shared__ uint32_t lval[kSortTile];
  const ClusterArgs &A = ctx.args();
  const uint64_t *__restrict__ pi = reinterpret_cast<const uint64_t *>(A.w.pass_info);
  const uint32_t *__restrict__ tile_off = A.w.tile_off;
  const uint32_t *__restrict__ digit_tot = A.w.hist_all;
  const int64_t tiles = A.w.sort_tiles;
  const uint64_t passes = pi[kPasses];
  if (static_cast<uint64_t>(pass) >= passes) return;
  const int64_t n = static_cast<int64_t>(pi[kNTotal]);
  // the in and out buffers of a pass are the two halves of one ping-pong pair
  const uint64_t *in = A.w.keys[pass & 1];
  const uint32_t *vin = A.w.vals[pass & 1];
  uint64_t *out = A.w.keys[(pass & 1) ^ 1];
  uint32_t *vout = A.w.vals[(pass & 1) ^ 1];
  const bool first = pass == 0, last = static_cast<uint64_t>(pass) + 1 == passes;
  const uint64_t kmin = pi[kMinKey], esc = pi[kEscKey];
  const int shift = 8 * pass;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t blk = ctx.block();
  const int64_t tile0 = blk * kSortTile;
  const int64_t rem = n - tile0;
  const int valid = rem < kSortTile ? static_cast<int>(rem) : kSortTile;

  for (int e = threadIdx.x; e < (DT / 64) * 256; e += DT) (&cnt[0][0])[e] = 0u;
  __syncthreads();

  const int64_t base = tile0 + w * (DSLOTS * 64);
  uint64_t key[DSLOTS];
  uint32_t val[DSLOTS], rank[DSLOTS];
  uint32_t dig[DSLOTS];
#pragma unroll
  for (int j = 0; j < DSLOTS; ++j) {
    const int64_t k = base + j * 64 + lane;
    const bool ok = k < n;
    key[j] = ok ? pass_key(in, k, first, kmin, esc) : 0ull;
    val[j] = ok ? (first ? static_cast<uint32_t>(k) : vin[k]) : 0u;
  }
#pragma unroll
  for (int j = 0; j < DSLOTS; ++j) {
    const bool ok = base + j * 64 + lane < n;
    const uint32_t d = static_cast<uint32_t>(key[j] >> shift) & 255u;
    dig[j] = ok ? d : 256u;
    // peers: valid lanes of this slot with the same digit
    uint64_t peers = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bal = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? bal : ~bal;
    }
    uint32_t before = 0u;
    if (ok) before = cnt[w][d];
    const uint32_t rk = static_cast<uint32_t>(__popcll(peers & lt));
    rank[j] = before + rk;
    __builtin_amdgcn_wave_barrier();
    if (ok && (peers & lt) == 0ull) cnt[w][d] = before + static_cast<uint32_t>(__popcll(peers));
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // Tile-local start of each digit and of each wave's share of it; gdelta
  // turns a tile-local position into the global one.
  {
    // threads 0..255 own one digit each; the rest add zeros to the scans
    const uint32_t d = threadIdx.x;
    const bool own = d < 256u;
    uint32_t tot = 0u;
    if (own)
      for (int q = 0; q < DT / 64; ++q) tot += cnt[q][d];
    const uint32_t lstart = block_excl_scan<DT>(tot, sh, static_cast<uint32_t *>(nullptr));
    const uint32_t dbase =
        block_excl_scan<DT>(own ? digit_tot[d] : 0u, sh, static_cast<uint32_t *>(nullptr));
    if (own) {
      gdelta[d] = dbase + tile_off[static_cast<int64_t>(d) * tiles + blk] - lstart;
      uint32_t acc = lstart;
      for (int q = 0; q < DT / 64; ++q) {
        const uint32_t c = cnt[q][d];
        cnt[q][d] = acc;
        acc += c;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < DSLOTS; ++j) {
    if (dig[j] < 256u) {
      const uint32_t lp = cnt[w][dig[j]] + rank[j];
      lkey[lp] = key[j];
      lval[lp] = val[j];
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < DSLOTS; ++j) {
    const int t = j * DT + threadIdx.x;
    if (t < valid) {
      const uint64_t kk = lkey[t];
      const uint32_t dst = gdelta[static_cast<uint32_t>(kk >> shift) & 255u] + t;
      if (!last) out[dst] = kk;
      vout[dst] = lval[t];
    }
  }
}

template <class Ctx, class Rec>
__global__ __launch_bounds__(NT) void k_gather(Ctx ctx, int normalise, int corr, int move_rng) {
  const ClusterArgs &A = ctx.args();
  const Rec *__restrict__ stage = static_cast<const Rec *>(A.w.stage);
  const uint32_t *__restrict__ vals0 = A.w.vals[0];
  const uint32_t *__restrict__ vals1 = A.w.vals[1];
  const uint64_t *__restrict__ pi = reinterpret_cast<const uint64_t *>(A.w.pass_info);
  const cmc_scalars *__restrict__ sc = A.s.sc;
  double *__restrict__ r = A.s.r;
  double *__restrict__ vr = A.s.vr;
  double *__restrict__ vt = A.s.vt;
  void *__restrict__ m = A.s.m;
  const int32_t m_f32 = A.s.m_f32;
  uint32_t *__restrict__ id = A.s.id;
  const int64_t kept = static_cast<int64_t>(pi[kNKept]);
  const int64_t p = ctx.block() * NT + threadIdx.x;
  if (p >= kept) return;
  const uint32_t *vals = (pi[kPasses] & 1ull) ? vals1 : vals0;
  const uint32_t src = pi[kPasses] ? vals[p] : static_cast<uint32_t>(p);
  const Rec rec = stage[src];
  r[p] = rec.r;
  vr[p] = rec.vr;
  vt[p] = rec.vt;
  const double mm = normalise ? static_cast<double>(rec.m) / sc->mass_norm
                              : static_cast<double>(rec.m);
  if (m_f32)
    static_cast<float *>(m)[p] = static_cast<float>(mm);
  else
    static_cast<double *>(m)[p] = mm;
  id[p] = rec.id;
  if (corr) A.w.perm[p] = src;
  if (move_rng && A.s.rng) store_lfsr(A.s.rng, p, A.w.rng_stage[src]);
}

// One thread per cluster: the device step counter moves on.
template <class Ctx>
__global__ void k_step_advance(Ctx ctx) {
  ctx.args().s.sc->step += 1;
}

}  // namespace

hipError_t launch_step_advance(const Target &t, hipStream_t st) {
  return dispatch(t, [&](const auto &l) {
    k_step_advance<<<l.grid(kShOne), 1, 0, st>>>(l.ctx(kShOne));
    return hipGetLastError();
  });
}

hipError_t launch_stage_from_state(const Target &t, bool, hipStream_t st) {
  return dispatch(t, [&](const auto &l) {
    k_stage_from_state<<<l.grid(kShStar), NT, 0, st>>>(l.ctx(kShStar));
    return hipGetLastError();
  });
}

// Sort the staged records by keys[0] (n = sc->n on entry) into the state.
hipError_t launch_sort_stage(const Target &t, bool m_f32, bool normalise_mass, bool step_records,
                             bool corr, bool move_rng, hipStream_t st) {
  const int c = corr ? 1 : 0, mv = move_rng ? 1 : 0;
  return dispatch(t, [&](const auto &l) {
    k_sort_prep<<<l.grid(kShOne), 1, 0, st>>>(l.ctx(kShOne));
    k_key_range<<<l.grid(kShKeyRange), NT, 0, st>>>(l.ctx(kShKeyRange));
    k_plan<<<l.grid(kShOne), NT, 0, st>>>(l.ctx(kShOne), c);
    for (int pass = 0; pass < 8; ++pass) {
      k_upsweep<<<l.grid(kShSortTile), NT, 0, st>>>(l.ctx(kShSortTile), pass);
      k_scan_digits<<<l.grid(kShDigit), NT, 0, st>>>(l.ctx(kShDigit), pass);
      k_downsweep<<<l.grid(kShSortTile), DT, 0, st>>>(l.ctx(kShSortTile), pass);
    }
    if (step_records && m_f32)
      k_gather<decltype(l.ctx(kShStar)), StageRec<float>>
          <<<l.grid(kShStar), NT, 0, st>>>(l.ctx(kShStar), normalise_mass ? 1 : 0, c, mv);
    else
      k_gather<decltype(l.ctx(kShStar)), WideRec>
          <<<l.grid(kShStar), NT, 0, st>>>(l.ctx(kShStar), normalise_mass ? 1 : 0, c, mv);
    return hipGetLastError();
  });
}

}  // namespace cmc

// rng.hip -- LFSR113 streams, the generator of arXiv:1206.5878 Sec. 3.6.
// The paper gives each processor its own stream of L'Ecuyer's combined
// Tausworthe generator by jumping D = 2^80 steps ahead from a seed state; here
// each star has one: star id's stream starts (base + id) * 2^80 steps in.
//
// A component step is linear over GF(2) in its 32-bit word, so n steps are
// the n-th power of a 32x32 bit matrix, held as its 32 columns (the image of
// each bit).  k_lfsr_tables squares each component's step matrix 80 times
// and keeps the powers 2^(80+b), b < 34; k_lfsr_seed multiplies a star's
// seed words by the powers of the bits of its stream index.
#include "cmc_internal.hpp"

namespace cmc {
namespace {

constexpr int NT = kBlock;
constexpr int kJumpSquarings = 80;  // log2 of the stream spacing D

__device__ __forceinline__ uint32_t taus_comp(int c, uint32_t z) {
  switch (c) {
    case 0: return taus_step<31, 6, 18>(z);
    case 1: return taus_step<29, 2, 2>(z);
    case 2: return taus_step<28, 13, 7>(z);
    default: return taus_step<25, 3, 13>(z);
  }
}

// M v over GF(2), M given by its columns.
__device__ __forceinline__ uint32_t mat_apply(const uint32_t *col, uint32_t v) {
  uint32_t r = 0u;
#pragma unroll 8
  for (int j = 0; j < 32; ++j) r ^= ((v >> j) & 1u) ? col[j] : 0u;
  return r;
}

// One block of 128 threads: thread (c, i) owns column i of component c.
__global__ __launch_bounds__(128) void k_lfsr_tables(uint32_t *__restrict__ table) {
  __shared__ uint32_t col[4][32];
  const int c = threadIdx.x >> 5, i = threadIdx.x & 31;
  col[c][i] = taus_comp(c, 1u << i);
  __syncthreads();
  for (int t = 0; t < kJumpSquarings + kLfsrStreamBits; ++t) {
    if (t >= kJumpSquarings)
      table[(c * kLfsrStreamBits + (t - kJumpSquarings)) * 32 + i] = col[c][i];
    const uint32_t sq = mat_apply(col[c], col[c][i]);  // M^2 e_i = M (M e_i)
    __syncthreads();
    col[c][i] = sq;
    __syncthreads();
  }
}

template <class Ctx>
__global__ __launch_bounds__(NT) void k_lfsr_seed(Ctx ctx, uint32_t z0, uint32_t z1, uint32_t z2,
                                                  uint32_t z3, uint64_t base) {
  __shared__ uint32_t tab[kLfsrJumpWords];
  const ClusterArgs &A = ctx.args();
  for (int q = threadIdx.x; q < kLfsrJumpWords; q += NT) tab[q] = A.w.lfsr_jump[q];
  __syncthreads();
  const int64_t j = ctx.block() * NT + threadIdx.x;
  if (j >= A.s.sc->n) return;
  const uint64_t sid = base + A.s.id[j];
  const uint32_t seed[4] = {z0, z1, z2, z3};
  Lfsr g;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    uint32_t v = seed[c];
    for (int b = 0; b < kLfsrStreamBits; ++b)
      if ((sid >> b) & 1u) v = mat_apply(tab + (c * kLfsrStreamBits + b) * 32, v);
    g.z[c] = v;
  }
  store_lfsr(A.s.rng, j, g);
}

__global__ __launch_bounds__(NT) void k_lfsr_words(const uint32_t *__restrict__ state,
                                                   uint32_t *__restrict__ out, int64_t n,
                                                   int32_t blocks) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
  if (i >= n) return;
  Lfsr g = load_lfsr(state, i);
  for (int32_t b = 0; b < blocks; ++b) {
    const U4 w = lfsr_block(g);
    uint32_t *o = out + 4 * (i * blocks + b);
    o[0] = w.x;
    o[1] = w.y;
    o[2] = w.z;
    o[3] = w.w;
  }
}

}  // namespace

hipError_t launch_lfsr_seed(const Target &t, const uint32_t z0[4], uint64_t stream_base,
                            hipStream_t st) {
  if (!t.one) return hipErrorInvalidValue;  // one cluster per call
  const OneL l{*t.one};
  k_lfsr_tables<<<1, 128, 0, st>>>(t.one->w.lfsr_jump);
  k_lfsr_seed<<<l.grid(kShStar), NT, 0, st>>>(l.ctx(kShStar), z0[0], z0[1], z0[2], z0[3],
                                              stream_base);
  return hipGetLastError();
}

hipError_t launch_lfsr_words(const uint32_t *state, uint32_t *out, int64_t n, int32_t blocks,
                             hipStream_t st) {
  if (n <= 0 || blocks <= 0) return hipSuccess;
  const unsigned grid = static_cast<unsigned>((n + NT - 1) / NT);
  k_lfsr_words<<<grid, NT, 0, st>>>(state, out, n, blocks);
  return hipGetLastError();
}

}  // namespace cmc

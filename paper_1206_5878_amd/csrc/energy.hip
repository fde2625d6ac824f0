// energy.hip -- the potential-change energy correction (arXiv:1206.5878,
// Sec. 2.1 item 6).  A step draws every orbit in the old potential Phi_old;
// once the stars have moved the potential is Phi_new.  Taking the potential
// to change linearly in time over the step, the work it does on a star that
// goes from r_old to r_new is the mean of dPhi = Phi_new - Phi_old at the two
// ends, while the drawn orbit already carries dPhi(r_new) into the new
// potential; so the kinetic energy per unit mass moves by
// dT = (dPhi(r_old) - dPhi(r_new)) / 2, applied by scaling vr and vt by one
// factor (their ratio is kept).
//
// The step's orbit pass records, in its own (staged) order, (r_old,
// Phi_old(r_old)) in cor and Phi_old(r_new) in pn; the sort records each
// sorted star's staged index in perm; sc->corr_n says how many stars were
// staged.  After the potential of the state the step left:
//   k_corr_old    staged order: pn_i += Phi_new(r_old_i) - Phi_old(r_old_i),
//                 Phi_new at the old radius from the new table, its interval
//                 through the radial index (the old radii are sorted, so
//                 neighbouring lanes search neighbouring buckets);
//   k_corr_apply  sorted order: dT = (pn[perm_j] - Phi_new(r_j)) / 2; the
//                 only random read is one 8-byte pn per star;
//   k_corr_done   nothing pending any more (standalone calls only: a step's
//                 sort sets sc->corr_n afresh).
#include "cmc_internal.hpp"

namespace cmc {
namespace {

constexpr int NT = kBlock;

template <class Ctx>
__global__ __launch_bounds__(NT) void k_corr_old(Ctx ctx) {
  const ClusterArgs &A = ctx.args();
  cmc_scalars *__restrict__ sc = A.s.sc;
  const int64_t np = sc->corr_n < A.s.cap ? sc->corr_n : A.s.cap;
  // every correction call reports its own skips, none when nothing is pending
  if (ctx.block() == 0 && threadIdx.x == 0) sc->corr_skipped = 0;
  if (np <= 0) return;
  const int64_t i = ctx.block() * NT + threadIdx.x;
  const RIndexCtl c = *A.w.rx_ctl;
  if (i >= np || c.n == 0) return;  // no star left: no new potential
  const RIndex ix{A.s.r, A.w.rx_start, A.w.rx_ctl};
  const RPhi o = A.w.cor[i];
  const int64_t k = rindex_last_le(ix, c, o.r);
  double phi_new;
  if (k < 0) {
    phi_new = A.w.lev[0][0].phi;  // inside the innermost star: flat
  } else {
    const MS t = A.w.ms[k];
    phi_new = -(t.M / o.r + t.S);
  }
  A.w.pn[i] = (phi_new - o.phi) + A.w.pn[i];
}

template <class Ctx>
__global__ __launch_bounds__(NT) void k_corr_apply(Ctx ctx) {
  const ClusterArgs &A = ctx.args();
  cmc_scalars *__restrict__ sc = A.s.sc;
  const int64_t np = sc->corr_n < A.s.cap ? sc->corr_n : A.s.cap, n = sc->n;
  if (np <= 0) return;
  const int64_t j = ctx.block() * NT + threadIdx.x;
  bool skip = false;
  if (j < n) {
    const uint32_t i = A.w.perm[j];
    if (i < np) {
      const double dT = 0.5 * (A.w.pn[i] - A.w.lev[0][j].phi);
      if (dT != 0.0) {
        const double vrj = A.s.vr[j], vtj = A.s.vt[j];
        const double v2 = vrj * vrj + vtj * vtj;
        if (v2 > 0.0 && v2 + 2.0 * dT > 0.0) {
          const double f = sqrt(1.0 + 2.0 * dT / v2);
          A.s.vr[j] = vrj * f;
          A.s.vt[j] = vtj * f;
        } else {
          skip = true;  // not enough kinetic energy (or none to scale)
        }
      }
    }
  }
  const uint64_t b = __ballot(skip);
  if ((threadIdx.x & 63) == 0 && b)
    atomicAdd(reinterpret_cast<unsigned long long *>(&sc->corr_skipped),
              static_cast<unsigned long long>(__popcll(b)));
}

template <class Ctx>
__global__ void k_corr_done(Ctx ctx) {
  ctx.args().s.sc->corr_n = 0;
}

}  // namespace

hipError_t launch_energy_correction(const Target &t, bool finish, hipStream_t st) {
  const hipError_t e = launch_rindex(t, st);
  if (e != hipSuccess) return e;
  return dispatch(t, [&](const auto &l) {
    k_corr_old<<<l.grid(kShStar), NT, 0, st>>>(l.ctx(kShStar));
    k_corr_apply<<<l.grid(kShStar), NT, 0, st>>>(l.ctx(kShStar));
    if (finish) k_corr_done<<<l.grid(kShOne), 1, 0, st>>>(l.ctx(kShOne));
    return hipGetLastError();
  });
}

}  // namespace cmc

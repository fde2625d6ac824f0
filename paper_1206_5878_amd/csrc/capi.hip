// capi.hip -- the extern "C" entry points of libcmc.so (declared in
// include/cmc.h): host-side argument checks, workspace carving, and the
// launch sequence of each step of arXiv:1206.5878 Sec. 2.1.  Nothing here
// allocates, frees or synchronises.
#include <mutex>

#include "cmc_internal.hpp"

using cmc::Workspace;

namespace cmc {

// ---------------------------------------------------------------- launch table
// Read-only while calls run (cmc_set_tuning is a setup call).  Built in: the
// autotuner's choices on an MI355X (tune.py, 5 timed steps per candidate):
// direct searches below 2^22 stars (the grouped form's sort costs more than
// it saves there), grouped ones above; larger trial chunks for larger N.
namespace {
constexpr cmc_tuning kBuiltinTuning[] = {
    {0, 0, 2048, 64, {0, 0, 0}},
    {int64_t(1) << 17, 0, 1024, 256, {0, 0, 0}},
    {int64_t(1) << 22, 1, 1024, 256, {0, 0, 0}},
};
cmc_tuning g_tuning[CMC_TUNING_MAX];
int32_t g_tuning_n = 0;  // 0: the built-in table
std::mutex g_tuning_mu;
}  // namespace

cmc_tuning tuning_for(int64_t cap) {
  const cmc_tuning *t = g_tuning_n ? g_tuning : kBuiltinTuning;
  const int32_t n = g_tuning_n ? g_tuning_n
                               : static_cast<int32_t>(sizeof(kBuiltinTuning) /
                                                      sizeof(kBuiltinTuning[0]));
  int32_t k = 0;
  while (k + 1 < n && t[k + 1].min_cap <= cap) ++k;
  return t[k];
}

// A capacity's launch settings into its workspace view.
void apply_tuning(Workspace &w, const cmc_tuning &t) {
  w.sorted = t.sorted;
  w.bracket_blocks = t.bracket_blocks;
  w.trial_chunk = t.trial_chunk;
}

ClusterArgs cluster_args(const cmc_state &s, uint64_t seed, double gamma) {
  ClusterArgs a{};
  a.s = s;
  a.w = layout(s.cap, s.work);
  apply_tuning(a.w, tuning_for(s.cap));
  a.top = orbit_top(a.w, s.cap);
  a.seed = seed;
  a.gamma = gamma;
  a.model = CMC_MODEL_PLUMMER;
  a.mass_spectrum = 0;
  a.w0 = 0.0;
  a.n_init = 0;
  a.bracket_blocks = blocks_of(kShBracket, a.w, s.cap);
  return a;
}

// potential (then the pending energy correction), timestep, relax, orbit,
// sort; events (if given) between them
hipError_t launch_step(const Target &t, bool m_f32, const cmc_params &p, void *const *events,
                       hipStream_t st) {
  auto mark = [&](int i) -> hipError_t {
    return events ? hipEventRecord(static_cast<hipEvent_t>(events[i]), st) : hipSuccess;
  };
  const bool corr = p.energy_corr != 0;
  hipError_t e = mark(0);
  if (e == hipSuccess) e = launch_potential(t, m_f32, p.precision, false, st);
  // the correction needs the radial index of the new radii, which the orbit
  // pass then reuses
  if (e == hipSuccess && corr) e = launch_energy_correction(t, false, st);
  if (e == hipSuccess) e = mark(1);
  if (e == hipSuccess) e = launch_timestep(t, m_f32, p, st);
  if (e == hipSuccess) e = mark(2);
  if (e == hipSuccess) e = launch_relax(t, m_f32, p, st);
  if (e == hipSuccess) e = mark(3);
  if (e == hipSuccess) e = launch_orbit(t, m_f32, p, true, corr, corr, st);
  if (e == hipSuccess) e = mark(4);
  if (e == hipSuccess) {
    e = bucket_sort_of(t) ? launch_bucket_sort(t, m_f32, corr, st)
                          : launch_sort_stage(t, m_f32, false, true, corr, true, st);
  }
  if (e == hipSuccess && p.step == CMC_STEP_DEVICE) e = launch_step_advance(t, st);
  if (e == hipSuccess) e = mark(5);
  return e;
}

}  // namespace cmc

static_assert(sizeof(cmc_scalars) == 128, "cmc_scalars is 128 bytes in the ABI");

namespace {

constexpr int64_t kMaxCap = (int64_t(1) << 31) - 1;  // table indices are 32-bit signed

int check_state(const cmc_state *s, Workspace *w) {
  if (!s || s->cap <= 0 || s->cap > kMaxCap) return CMC_EINVAL;
  if (!s->r || !s->vr || !s->vt || !s->m || !s->id || !s->phi || !s->mcum || !s->ssuf ||
      !s->r_new || !s->sc || !s->work)
    return CMC_EINVAL;
  if (reinterpret_cast<uintptr_t>(s->work) % 256 != 0) return CMC_EINVAL;
  *w = cmc::layout(s->cap, s->work);
  if (s->work_bytes < w->bytes) return CMC_EWORKSPACE;
  return CMC_OK;
}

int check_params(const cmc_params *p) {
  if (!p) return CMC_EINVAL;
  if (p->precision != CMC_FP64 && p->precision != CMC_MIXED) return CMC_EINVAL;
  if (!(p->gamma > 0.0) || !(p->target > 0.0 && p->target < 1.0)) return CMC_EINVAL;
  if (p->bound_factor < 0.0 || p->trial_cap < 0 || p->dt_iters < 0) return CMC_EINVAL;
  if (p->energy_corr != 0 && p->energy_corr != 1) return CMC_EINVAL;
  if (p->rng != CMC_RNG_PHILOX && p->rng != CMC_RNG_LFSR113) return CMC_EINVAL;
  return CMC_OK;
}

// A step, timestep, relaxation or orbit call that draws from LFSR113 streams
// needs the state's stream array.
int check_rng(const cmc_state *s, const cmc_params *p) {
  return (p->rng == CMC_RNG_LFSR113 && !s->rng) ? CMC_EINVAL : CMC_OK;
}

int status_of(hipError_t e) { return e == hipSuccess ? CMC_OK : CMC_EHIP; }

// The launch target of a single-cluster call.
struct Single {
  cmc::ClusterArgs a;
  cmc::Target t() const { return cmc::Target{&a, nullptr}; }
};
Single single(const cmc_state &s, uint64_t seed, double gamma) {
  return Single{cmc::cluster_args(s, seed, gamma)};
}

hipStream_t as_stream(void *stream) { return static_cast<hipStream_t>(stream); }

// ---------------------------------------------------------------- static scratch
// The workspace of cmc_step_noalloc: one copy per GPU, for the whole process.
// In host code `scratch` names a host-side stand-in, not device memory: only
// the address hipGetSymbolAddress returns for the current device is passed on.
__device__ __align__(256) unsigned char scratch[CMC_SCRATCH_BYTES];

constexpr int kScratchDevices = 64;
std::mutex scratch_mu;
void *scratch_addr[kScratchDevices];  // device address of `scratch`, per device

// The current device's scratch address, looked up on the first call made
// while that device is current.
int scratch_of_current_device(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return CMC_EHIP;
  if (dev < 0 || dev >= kScratchDevices) return CMC_EINVAL;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_addr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CMC_EHIP;
    if (reinterpret_cast<uintptr_t>(p) % 256 != 0) return CMC_EHIP;
    scratch_addr[dev] = p;
  }
  *out = scratch_addr[dev];
  return CMC_OK;
}

}  // namespace

extern "C" {

int cmc_abi_version(void) { return CMC_ABI_VERSION; }

int cmc_set_tuning(const cmc_tuning *entries, int32_t n) {
  if (n < 0 || n > CMC_TUNING_MAX || (n > 0 && !entries)) return CMC_EINVAL;
  for (int32_t k = 0; k < n; ++k) {
    const cmc_tuning &t = entries[k];
    if (k == 0 ? t.min_cap != 0 : t.min_cap <= entries[k - 1].min_cap) return CMC_EINVAL;
    if (t.sorted != 0 && t.sorted != 1) return CMC_EINVAL;
    if (t.bracket_blocks < 8 || t.bracket_blocks > 65535) return CMC_EINVAL;
    if (t.trial_chunk < 64 || t.trial_chunk > 1024 || t.trial_chunk % 64 != 0) return CMC_EINVAL;
  }
  std::lock_guard<std::mutex> lock(cmc::g_tuning_mu);
  for (int32_t k = 0; k < n; ++k) cmc::g_tuning[k] = entries[k];
  cmc::g_tuning_n = n;
  return CMC_OK;
}

int cmc_get_tuning(int64_t cap, cmc_tuning *out) {
  if (!out || cap < 0) return CMC_EINVAL;
  *out = cmc::tuning_for(cap);
  return CMC_OK;
}

size_t cmc_workspace_bytes(int64_t cap) {
  if (cap <= 0 || cap > kMaxCap) return 0;
  return cmc::layout(cap, nullptr).bytes;
}

const char *cmc_strerror(int code) {
  switch (code) {
    case CMC_OK:
      return "ok";
    case CMC_EINVAL:
      return "invalid argument (null pointer, capacity out of range, bad parameter)";
    case CMC_EWORKSPACE:
      return "workspace smaller than cmc_workspace_bytes(cap)";
    case CMC_EHIP:
      return "HIP kernel launch failed";
    case CMC_ERANGE:
      return "star count larger than the state capacity";
    case CMC_ESCRATCH:
      return "capacity too large for the library's static scratch (CMC_SCRATCH_BYTES)";
    default:
      return "unknown cmc error code";
  }
}

int cmc_init_model(cmc_state *s, int64_t n, uint64_t seed, int32_t model, int32_t mass_spectrum,
                   double w0, void *stream) {
  Workspace w;
  int rc = check_state(s, &w);
  if (rc) return rc;
  if (n < 0) return CMC_EINVAL;
  if (n > s->cap) return CMC_ERANGE;
  if (mass_spectrum != 0 && mass_spectrum != 1) return CMC_EINVAL;
  if (model != CMC_MODEL_PLUMMER && model != CMC_MODEL_KING) return CMC_EINVAL;
  if (model == CMC_MODEL_KING && !(w0 > 0.0 && w0 <= 16.0)) return CMC_EINVAL;
  Single one = single(*s, seed, 1.0);
  one.a.model = model;
  one.a.mass_spectrum = mass_spectrum;
  one.a.w0 = w0;
  one.a.n_init = n;
  return status_of(cmc::launch_init(one.t(), s->m_f32 != 0, as_stream(stream)));
}

int cmc_init_plummer(cmc_state *s, int64_t n, uint64_t seed, int32_t mass_spectrum,
                     void *stream) {
  return cmc_init_model(s, n, seed, CMC_MODEL_PLUMMER, mass_spectrum, 0.0, stream);
}

int cmc_sort(cmc_state *s, void *stream) {
  Workspace w;
  int rc = check_state(s, &w);
  if (rc) return rc;
  const Single one = single(*s, 0, 1.0);
  hipError_t e = cmc::launch_stage_from_state(one.t(), s->m_f32 != 0, as_stream(stream));
  if (e != hipSuccess) return CMC_EHIP;
  return status_of(
      cmc::launch_sort_stage(one.t(), s->m_f32 != 0, false, false, false, true,
                             as_stream(stream)));
}

int cmc_potential(cmc_state *s, int32_t precision, void *stream) {
  Workspace w;
  int rc = check_state(s, &w);
  if (rc) return rc;
  if (precision != CMC_FP64 && precision != CMC_MIXED) return CMC_EINVAL;
  const Single one = single(*s, 0, 1.0);
  return status_of(
      cmc::launch_potential(one.t(), s->m_f32 != 0, precision, true, as_stream(stream)));
}

int cmc_timestep(cmc_state *s, const cmc_params *p, void *stream) {
  Workspace w;
  int rc = check_state(s, &w);
  if (rc) return rc;
  if ((rc = check_params(p))) return rc;
  if ((rc = check_rng(s, p))) return rc;
  const Single one = single(*s, p->seed, p->gamma);
  return status_of(cmc::launch_timestep(one.t(), s->m_f32 != 0, *p, as_stream(stream)));
}

int cmc_relax(cmc_state *s, const cmc_params *p, void *stream) {
  Workspace w;
  int rc = check_state(s, &w);
  if (rc) return rc;
  if ((rc = check_params(p))) return rc;
  if ((rc = check_rng(s, p))) return rc;
  const Single one = single(*s, p->seed, p->gamma);
  return status_of(cmc::launch_relax(one.t(), s->m_f32 != 0, *p, as_stream(stream)));
}

int cmc_orbit(cmc_state *s, const cmc_params *p, void *stream) {
  Workspace w;
  int rc = check_state(s, &w);
  if (rc) return rc;
  if ((rc = check_params(p))) return rc;
  if ((rc = check_rng(s, p))) return rc;
  const Single one = single(*s, p->seed, p->gamma);
  hipError_t e = cmc::launch_table_pack(one.t(), as_stream(stream));
  if (e == hipSuccess)
    e = cmc::launch_orbit(one.t(), s->m_f32 != 0, *p, false, false, false, as_stream(stream));
  return status_of(e);
}

// The step's five phases; events (if given) are recorded between them.
static int run_step(cmc_state *s, const cmc_params *p, void *const *events, hipStream_t st) {
  Workspace w;
  int rc = check_state(s, &w);
  if (rc) return rc;
  if ((rc = check_params(p))) return rc;
  if ((rc = check_rng(s, p))) return rc;
  const Single one = single(*s, p->seed, p->gamma);
  return status_of(cmc::launch_step(one.t(), s->m_f32 != 0, *p, events, st));
}

int cmc_step(cmc_state *s, const cmc_params *p, void *stream) {
  return run_step(s, p, nullptr, as_stream(stream));
}

int cmc_step_noalloc(cmc_state *s, const cmc_params *p, void *stream) {
  if (!s || s->cap <= 0 || s->cap > kMaxCap) return CMC_EINVAL;
  if (cmc::layout(s->cap, nullptr).bytes > CMC_SCRATCH_BYTES) return CMC_ESCRATCH;
  int rc = check_params(p);
  if (rc) return rc;
  if (p->energy_corr != 0) return CMC_EINVAL;
  void *ptr = nullptr;
  if ((rc = scratch_of_current_device(&ptr))) return rc;
  cmc_state t = *s;
  t.work = ptr;
  t.work_bytes = CMC_SCRATCH_BYTES;
  return run_step(&t, p, nullptr, as_stream(stream));
}

int cmc_step_timed(cmc_state *s, const cmc_params *p, void *const *events, void *stream) {
  if (!events) return CMC_EINVAL;
  for (int i = 0; i < 6; ++i)
    if (!events[i]) return CMC_EINVAL;
  return run_step(s, p, events, as_stream(stream));
}

int cmc_energy_correction(cmc_state *s, void *stream) {
  Workspace w;
  int rc = check_state(s, &w);
  if (rc) return rc;
  const Single one = single(*s, 0, 1.0);
  return status_of(cmc::launch_energy_correction(one.t(), true, as_stream(stream)));
}

int cmc_diagnostics(const cmc_state *s, double *out_dev, void *stream) {
  Workspace w;
  int rc = check_state(s, &w);
  if (rc) return rc;
  if (!out_dev) return CMC_EINVAL;
  const Single one = single(*s, 0, 1.0);
  return status_of(cmc::launch_diagnostics(one.t(), s->m_f32 != 0, out_dev, as_stream(stream)));
}

int cmc_philox(uint64_t key, const uint32_t *ctr_dev, uint32_t *out_dev, int64_t n,
               void *stream) {
  if (n < 0 || (n > 0 && (!ctr_dev || !out_dev))) return CMC_EINVAL;
  return status_of(cmc::launch_philox(key, ctr_dev, out_dev, n, as_stream(stream)));
}

int cmc_rng_seed_lfsr113(cmc_state *s, const uint32_t *z0, uint64_t stream_base, void *stream) {
  Workspace w;
  int rc = check_state(s, &w);
  if (rc) return rc;
  if (!s->rng || !z0 || stream_base >= (uint64_t(1) << 33)) return CMC_EINVAL;
  // each component needs a nonzero state in its top k bits (k = 31, 29, 28, 25)
  if (z0[0] < 2u || z0[1] < 8u || z0[2] < 16u || z0[3] < 128u) return CMC_EINVAL;
  const uint32_t z[4] = {z0[0], z0[1], z0[2], z0[3]};
  const Single one = single(*s, 0, 1.0);
  return status_of(cmc::launch_lfsr_seed(one.t(), z, stream_base, as_stream(stream)));
}

int cmc_lfsr113(const uint32_t *state_dev, uint32_t *out_dev, int64_t n, int32_t blocks,
                void *stream) {
  if (n < 0 || blocks < 0 || (n > 0 && blocks > 0 && (!state_dev || !out_dev)))
    return CMC_EINVAL;
  return status_of(cmc::launch_lfsr_words(state_dev, out_dev, n, blocks, as_stream(stream)));
}

}  // extern "C"

// batch.hip -- ensembles: many independent clusters advanced by the same
// launches.  Each cluster keeps its own state arrays and workspace; one
// device table holds every cluster's arguments (ClusterArgs), and for every
// launch shape a map from the launch's blocks to (cluster, block of the
// cluster).  Every kernel of the single-cluster path runs unchanged on top
// of that (the Many launch context), so per-cluster scans, reductions,
// timestep solves and sorts never cross a cluster.
#include <algorithm>
#include <cmath>
#include <vector>

#include "cmc_internal.hpp"

namespace cmc {
namespace {

constexpr int kMaxClusters = 65535;  // the block maps are 16-bit
static_assert(kShapes <= CMC_SHAPES, "launch shapes fit the handle");

struct BatchLayout {
  size_t args, first, map[kShapes], bytes;
};

BatchLayout batch_layout(int32_t clusters, const int64_t *total) {
  BatchLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = (off + 255) & ~size_t(255);
    const size_t at = off;
    off += bytes;
    return at;
  };
  L.args = take(sizeof(ClusterArgs) * clusters);
  L.first = take(sizeof(int64_t) * kShapes * (clusters + 1));
  for (int sh = 0; sh < kShapes; ++sh) L.map[sh] = take(sizeof(uint16_t) * total[sh]);
  L.bytes = (off + 255) & ~size_t(255);
  return L;
}

// Blocks of each cluster in each launch shape.  The bracket kernel's
// resident blocks (the launch table's entry for the largest capacity) go to
// the largest cluster, and to each other cluster in proportion to its
// capacity: every cluster gets the density of resident blocks the entry
// gives the largest one (at 64 clusters from 1e4 to 9.4e5 stars, 5.47 ms a
// step against 5.83 ms for the same blocks shared out over the summed
// capacity).
void shape_blocks(const std::vector<ClusterArgs> &a, std::vector<int64_t> *blocks) {
  const int C = static_cast<int>(a.size());
  double cap_max = 1.0;
  for (const auto &x : a) cap_max = std::max(cap_max, static_cast<double>(x.s.cap));
  const int64_t resident = a.empty() ? 1 : a[0].w.bracket_blocks;
  for (int sh = 0; sh < kShapes; ++sh) {
    blocks[sh].assign(C, 0);
    for (int c = 0; c < C; ++c) {
      const Workspace &w = a[c].w;
      int64_t b = blocks_of(static_cast<Shape>(sh), w, a[c].s.cap);
      if (sh == kShBracket) {
        const int64_t share = static_cast<int64_t>(
            std::llround(resident * static_cast<double>(a[c].s.cap) / cap_max));
        b = std::max<int64_t>(1, std::min<int64_t>(share, b));
      }
      blocks[sh][c] = b;
    }
  }
}

int check_state(const cmc_state &s) {
  if (s.cap <= 0 || s.cap > (int64_t(1) << 31) - 1) return CMC_EINVAL;
  if (!s.r || !s.vr || !s.vt || !s.m || !s.id || !s.phi || !s.mcum || !s.ssuf || !s.r_new ||
      !s.sc || !s.work)
    return CMC_EINVAL;
  if (reinterpret_cast<uintptr_t>(s.work) % 256 != 0) return CMC_EINVAL;
  if (s.work_bytes < layout(s.cap, nullptr).bytes) return CMC_EWORKSPACE;
  return CMC_OK;
}

int totals(const cmc_state *states, int32_t clusters, std::vector<ClusterArgs> *args,
           std::vector<int64_t> *blocks, int64_t *total) {
  if (!states || clusters < 1 || clusters > kMaxClusters) return CMC_EINVAL;
  args->clear();
  int64_t cap_max = 0;
  for (int c = 0; c < clusters; ++c) {
    const int rc = check_state(states[c]);
    if (rc) return rc;
    if ((states[c].m_f32 != 0) != (states[0].m_f32 != 0)) return CMC_EINVAL;
    args->push_back(cluster_args(states[c], 0, 1.0));
    cap_max = states[c].cap > cap_max ? states[c].cap : cap_max;
  }
  // one launch table entry for the whole ensemble: that of its largest
  // cluster, since the searches run on each cluster's own table (64 clusters
  // of 1e4..1e6 stars, 1.4e7 in all: the direct form, 6.02 ms per step,
  // against 6.36 ms with the grouped form that the summed capacity's entry
  // names)
  const cmc_tuning tun = tuning_for(cap_max);
  for (auto &a : *args) apply_tuning(a.w, tun);
  shape_blocks(*args, blocks);
  for (int sh = 0; sh < kShapes; ++sh) {
    int64_t t = 0;
    for (int c = 0; c < clusters; ++c) t += blocks[sh][c];
    if (t > 0x7fffffff) return CMC_ERANGE;  // a grid's block count
    total[sh] = t;
  }
  return CMC_OK;
}

BatchDev batch_dev(const cmc_batch &b) {
  BatchDev d{};
  int64_t total[kShapes];
  for (int sh = 0; sh < kShapes; ++sh) total[sh] = b.total[sh];
  const BatchLayout L = batch_layout(b.clusters, total);
  char *base = static_cast<char *>(b.dev);
  d.clusters = b.clusters;
  d.args = reinterpret_cast<const ClusterArgs *>(base + L.args);
  for (int sh = 0; sh < kShapes; ++sh) {
    d.first[sh] = reinterpret_cast<const int64_t *>(base + L.first) + sh * (b.clusters + 1);
    d.map[sh] = reinterpret_cast<const uint16_t *>(base + L.map[sh]);
    d.total[sh] = b.total[sh];
  }
  d.top_entries = b.top_entries;
  d.any_f32 = b.m_f32;
  d.any_f64 = !b.m_f32;
  d.bucket_sort = b.bucket_sort;
  d.sorted = b.sorted_searches;
  return d;
}

int check_batch(const cmc_batch *b) {
  if (!b || !b->dev || b->clusters < 1 || b->clusters > kMaxClusters) return CMC_EINVAL;
  int64_t total[kShapes];
  for (int sh = 0; sh < kShapes; ++sh) total[sh] = b->total[sh];
  if (b->dev_bytes < batch_layout(b->clusters, total).bytes) return CMC_EWORKSPACE;
  return CMC_OK;
}

// The step parameters an ensemble call reads (seed and gamma come from each
// cluster's spec instead).
int check_batch_params(const cmc_batch *b, const cmc_params *p) {
  if (!p || (p->precision != CMC_FP64 && p->precision != CMC_MIXED)) return CMC_EINVAL;
  if (!(p->target > 0.0 && p->target < 1.0)) return CMC_EINVAL;
  if (p->bound_factor < 0.0 || p->trial_cap < 0 || p->dt_iters < 0) return CMC_EINVAL;
  if (p->energy_corr != 0 && p->energy_corr != 1) return CMC_EINVAL;
  if (p->rng != CMC_RNG_PHILOX && p->rng != CMC_RNG_LFSR113) return CMC_EINVAL;
  if (p->rng == CMC_RNG_LFSR113 && !b->lfsr_ready) return CMC_EINVAL;
  return CMC_OK;
}

int status_of(hipError_t e) { return e == hipSuccess ? CMC_OK : CMC_EHIP; }

}  // namespace
}  // namespace cmc

extern "C" {

size_t cmc_batch_device_bytes(const cmc_state *states, int32_t clusters) {
  std::vector<cmc::ClusterArgs> args;
  std::vector<int64_t> blocks[cmc::kShapes];
  int64_t total[cmc::kShapes];
  if (cmc::totals(states, clusters, &args, blocks, total)) return 0;
  return cmc::batch_layout(clusters, total).bytes;
}

int cmc_batch_prepare(cmc_batch *b, const cmc_state *states, const cmc_cluster_spec *specs,
                      int32_t clusters, void *dev, size_t dev_bytes) {
  if (!b || !specs || !dev || reinterpret_cast<uintptr_t>(dev) % 256 != 0) return CMC_EINVAL;
  std::vector<cmc::ClusterArgs> args;
  std::vector<int64_t> blocks[cmc::kShapes];
  int64_t total[cmc::kShapes];
  int rc = cmc::totals(states, clusters, &args, blocks, total);
  if (rc) return rc;
  const cmc::BatchLayout L = cmc::batch_layout(clusters, total);
  if (dev_bytes < L.bytes) return CMC_EWORKSPACE;
  int32_t top = 0, bucket = 1, lfsr = 1;
  for (int c = 0; c < clusters; ++c) {
    const cmc_cluster_spec &sp = specs[c];
    if (sp.n < 0) return CMC_EINVAL;
    if (sp.n > states[c].cap) return CMC_ERANGE;
    if (!(sp.gamma > 0.0)) return CMC_EINVAL;
    if (sp.model != CMC_MODEL_PLUMMER && sp.model != CMC_MODEL_KING) return CMC_EINVAL;
    if (sp.model == CMC_MODEL_KING && !(sp.w0 > 0.0 && sp.w0 <= 16.0)) return CMC_EINVAL;
    if (sp.mass_spectrum != 0 && sp.mass_spectrum != 1) return CMC_EINVAL;
    cmc::ClusterArgs &a = args[c];
    a.seed = sp.seed;
    a.gamma = sp.gamma;
    a.model = sp.model;
    a.mass_spectrum = sp.mass_spectrum;
    a.w0 = sp.w0;
    a.n_init = sp.n;
    a.bracket_blocks = blocks[cmc::kShBracket][c];
    top = std::max(top, a.top.entries);
    if (a.w.bkt_bins == 0) bucket = 0;
    if (!states[c].rng) lfsr = 0;
  }
  // tables: arguments, first block of each cluster per shape, block maps
  std::vector<char> host(L.bytes, 0);
  std::copy(reinterpret_cast<const char *>(args.data()),
            reinterpret_cast<const char *>(args.data() + clusters), host.data() + L.args);
  int64_t *first = reinterpret_cast<int64_t *>(host.data() + L.first);
  for (int sh = 0; sh < cmc::kShapes; ++sh) {
    int64_t at = 0;
    uint16_t *map = reinterpret_cast<uint16_t *>(host.data() + L.map[sh]);
    for (int c = 0; c < clusters; ++c) {
      first[sh * (clusters + 1) + c] = at;
      for (int64_t k = 0; k < blocks[sh][c]; ++k) map[at + k] = static_cast<uint16_t>(c);
      at += blocks[sh][c];
    }
    first[sh * (clusters + 1) + clusters] = at;
  }
  if (hipMemcpy(dev, host.data(), L.bytes, hipMemcpyHostToDevice) != hipSuccess) return CMC_EHIP;
  b->clusters = clusters;
  b->m_f32 = states[0].m_f32 != 0;
  b->dev = dev;
  b->dev_bytes = dev_bytes;
  for (int sh = 0; sh < CMC_SHAPES; ++sh) b->total[sh] = sh < cmc::kShapes ? total[sh] : 0;
  b->top_entries = top;
  b->bucket_sort = bucket;
  b->lfsr_ready = lfsr;
  b->sorted_searches = args[0].w.sorted;
  return CMC_OK;
}

int cmc_batch_init(const cmc_batch *b, void *stream) {
  int rc = cmc::check_batch(b);
  if (rc) return rc;
  const cmc::BatchDev d = cmc::batch_dev(*b);
  return cmc::status_of(cmc::launch_init(cmc::Target{nullptr, &d}, b->m_f32 != 0,
                                         static_cast<hipStream_t>(stream)));
}

int cmc_batch_step(const cmc_batch *b, const cmc_params *p, void *stream) {
  int rc = cmc::check_batch(b);
  if (rc) return rc;
  if ((rc = cmc::check_batch_params(b, p))) return rc;
  const cmc::BatchDev d = cmc::batch_dev(*b);
  return cmc::status_of(cmc::launch_step(cmc::Target{nullptr, &d}, b->m_f32 != 0, *p, nullptr,
                                         static_cast<hipStream_t>(stream)));
}

int cmc_batch_sort(const cmc_batch *b, void *stream) {
  int rc = cmc::check_batch(b);
  if (rc) return rc;
  const cmc::BatchDev d = cmc::batch_dev(*b);
  const cmc::Target t{nullptr, &d};
  const hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = cmc::launch_stage_from_state(t, b->m_f32 != 0, st);
  if (e == hipSuccess) e = cmc::launch_sort_stage(t, b->m_f32 != 0, false, false, false, true, st);
  return cmc::status_of(e);
}

int cmc_batch_timestep(const cmc_batch *b, const cmc_params *p, void *stream) {
  int rc = cmc::check_batch(b);
  if (rc) return rc;
  if ((rc = cmc::check_batch_params(b, p))) return rc;
  const cmc::BatchDev d = cmc::batch_dev(*b);
  return cmc::status_of(cmc::launch_timestep(cmc::Target{nullptr, &d}, b->m_f32 != 0, *p,
                                             static_cast<hipStream_t>(stream)));
}

int cmc_batch_relax(const cmc_batch *b, const cmc_params *p, void *stream) {
  int rc = cmc::check_batch(b);
  if (rc) return rc;
  if ((rc = cmc::check_batch_params(b, p))) return rc;
  const cmc::BatchDev d = cmc::batch_dev(*b);
  return cmc::status_of(cmc::launch_relax(cmc::Target{nullptr, &d}, b->m_f32 != 0, *p,
                                          static_cast<hipStream_t>(stream)));
}

int cmc_batch_orbit(const cmc_batch *b, const cmc_params *p, void *stream) {
  int rc = cmc::check_batch(b);
  if (rc) return rc;
  if ((rc = cmc::check_batch_params(b, p))) return rc;
  const cmc::BatchDev d = cmc::batch_dev(*b);
  const cmc::Target t{nullptr, &d};
  const hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = cmc::launch_table_pack(t, st);
  if (e == hipSuccess) e = cmc::launch_orbit(t, b->m_f32 != 0, *p, false, false, false, st);
  return cmc::status_of(e);
}

int cmc_batch_potential(const cmc_batch *b, int32_t precision, void *stream) {
  int rc = cmc::check_batch(b);
  if (rc) return rc;
  if (precision != CMC_FP64 && precision != CMC_MIXED) return CMC_EINVAL;
  const cmc::BatchDev d = cmc::batch_dev(*b);
  return cmc::status_of(cmc::launch_potential(cmc::Target{nullptr, &d}, b->m_f32 != 0,
                                              precision, true, static_cast<hipStream_t>(stream)));
}

int cmc_batch_energy_correction(const cmc_batch *b, void *stream) {
  int rc = cmc::check_batch(b);
  if (rc) return rc;
  const cmc::BatchDev d = cmc::batch_dev(*b);
  return cmc::status_of(cmc::launch_energy_correction(cmc::Target{nullptr, &d}, true,
                                                      static_cast<hipStream_t>(stream)));
}

int cmc_batch_diagnostics(const cmc_batch *b, double *out_dev, void *stream) {
  int rc = cmc::check_batch(b);
  if (rc) return rc;
  if (!out_dev) return CMC_EINVAL;
  const cmc::BatchDev d = cmc::batch_dev(*b);
  return cmc::status_of(cmc::launch_diagnostics(cmc::Target{nullptr, &d}, b->m_f32 != 0,
                                                out_dev, static_cast<hipStream_t>(stream)));
}

}  // extern "C"

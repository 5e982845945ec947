// api.cpp -- the C ABI of the photon-transport library (declared in
// include/xephot.h): context, validation, optical tables, BVH upload, launches
// and the launch-configuration autotuner.  No exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "xp_internal.h"

struct xp_context {
  int device = 0;
  int n_cu = 0;
  size_t max_lds = 0;
  std::string err;
  // mesh (host copy)
  bool mesh_loaded = false;
  std::vector<float> vtx;
  std::vector<int32_t> tri, mat_in, mat_out, surf, sensor;
  int32_t max_mat = -1, max_surf = -1, max_sensor = -1;
  // tables
  std::vector<xp_material> mats;
  std::vector<std::vector<std::array<float, 4>>> disp;  // per material: (lambda, n, L_abs, L_R)
  std::vector<xp_surface> surfs;
  std::vector<int32_t> channel;
  int32_t n_channels = 0;
  bool channel_set = false;
  // device state
  bool bvh_built = false;
  xp::BvhResult bvh;
  xp_bvh_info stats{};
  xp::Node4* d_nodes = nullptr;
  xp::TriRec* d_tris = nullptr;
  int32_t* d_channel = nullptr;
  int32_t d_channel_len = 0;
  int32_t* d_tri_group = nullptr;       // loss group per mesh triangle
  int32_t n_groups = 0;                 // 0: no loss groups set
  unsigned long long* d_counters = nullptr;        // ring of kCounterRing eager-launch counters
  unsigned long long* d_graph_counters = nullptr;  // one per launch captured in a graph
  int32_t graph_next = 0;                          // graph counters handed out
  int32_t* d_stack_overflow = nullptr;  // per-lane spill slots of the traversal stack
  int64_t stack_overflow_lanes = 0;
  unsigned ring_next = 0;
  bool tuned = false;
  xp_launch_cfg tuned_cfg{};
};

namespace {

thread_local std::string g_thread_err;

int fail(xp_context* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  g_thread_err = msg;
  return code;
}

int hip_fail(xp_context* ctx, hipError_t e, const char* what) {
  return fail(ctx, e == hipErrorOutOfMemory ? XP_ERR_OOM : XP_ERR_HIP,
              std::string(what) + ": " + hipGetErrorString(e));
}

struct DeviceGuard {
  int old = -1;
  hipError_t status = hipSuccess;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&old) != hipSuccess) old = -1;
    if (old != dev) status = hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (old >= 0 && hipGetDevice(&cur) == hipSuccess && cur != old) (void)hipSetDevice(old);
  }
};

template <class T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

bool finite_pos(float x) { return std::isfinite(x) && x > 0.0f; }

int upload_channel_map(xp_context* ctx) {
  std::vector<int32_t> map;
  int32_t nch;
  if (ctx->channel_set) {
    map = ctx->channel;
    nch = ctx->n_channels;
  } else {
    const int32_t ns = std::max(ctx->max_sensor + 1, 1);
    map.resize(ns);
    for (int32_t i = 0; i < ns; ++i) map[i] = i;
    nch = ns;
  }
  if (map.empty()) map.push_back(0);
  dfree(ctx->d_channel);
  hipError_t e = hipMalloc(&ctx->d_channel, map.size() * sizeof(int32_t));
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMalloc(channel map)");
  e = hipMemcpy(ctx->d_channel, map.data(), map.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpy(channel map)");
  ctx->d_channel_len = int32_t(map.size());
  ctx->n_channels = nch;
  return XP_OK;
}

xp_launch_cfg default_cfg() {
  return xp_launch_cfg{256, 0, 64, -1, xp::kStackLds, xp::kWaveBatch, 0};
}

// Validates (ctx, src, rp) for a launch and fills the kernel arguments.
int prepare(xp_context* ctx, const xp_sources* src, const xp_run_params* rp,
            const xp_launch_cfg* lc_in, xp::LaunchArgs& a, xp_launch_cfg& lc, int& grid) {
  if (!ctx) return fail(nullptr, XP_ERR_INVALID_ARG, "null context");
  if (!src || !rp) return fail(ctx, XP_ERR_INVALID_ARG, "null sources or run parameters");
  if (!ctx->bvh_built) return fail(ctx, XP_ERR_STATE, "xp_build_bvh has not been called");
  if (int32_t(ctx->mats.size()) <= ctx->max_mat)
    return fail(ctx, XP_ERR_STATE, "material table does not cover the mesh's material ids");
  if (int32_t(ctx->surfs.size()) <= ctx->max_surf)
    return fail(ctx, XP_ERR_STATE, "surface table does not cover the mesh's surface ids");
  if (ctx->channel_set && int32_t(ctx->channel.size()) <= ctx->max_sensor)
    return fail(ctx, XP_ERR_STATE, "channel map does not cover the mesh's sensor ids");
  if (src->n_photons < 0) return fail(ctx, XP_ERR_INVALID_ARG, "n_photons < 0");
  if (src->medium < 0 || src->medium >= int32_t(ctx->mats.size()))
    return fail(ctx, XP_ERR_INVALID_ARG, "source medium is not a material id");
  if (rp->grad_material < -1 || rp->grad_material >= int32_t(ctx->mats.size()))
    return fail(ctx, XP_ERR_INVALID_ARG, "grad_material out of range");
  if (!(rp->eps >= 0.0f) || !std::isfinite(rp->eps))
    return fail(ctx, XP_ERR_INVALID_ARG, "eps must be finite and >= 0");
  if (!(rp->surface_offset >= 0.0f) || !(rp->surface_offset < 1e-2f))
    return fail(ctx, XP_ERR_INVALID_ARG, "surface_offset must be in [0, 1e-2) m");
  switch (src->kind) {
    case XP_SRC_POINTS:
      if (!src->positions || src->n_sources <= 0)
        return fail(ctx, XP_ERR_INVALID_ARG, "POINTS needs positions and n_sources > 0");
      if (!src->offsets) {
        if (src->count_per_source <= 0)
          return fail(ctx, XP_ERR_INVALID_ARG, "POINTS without offsets needs count_per_source > 0");
        if (src->n_photons > src->n_sources * src->count_per_source)
          return fail(ctx, XP_ERR_INVALID_ARG, "n_photons exceeds n_sources * count_per_source");
      }
      if (src->per_source_events && src->n_sources > INT32_MAX)
        return fail(ctx, XP_ERR_INVALID_ARG, "too many events");
      break;
    case XP_SRC_UNIFORM_CYLINDER:
      if (!finite_pos(src->cyl_radius) || !std::isfinite(src->cyl_zlo) ||
          !std::isfinite(src->cyl_zhi) || src->cyl_zhi < src->cyl_zlo)
        return fail(ctx, XP_ERR_INVALID_ARG, "bad cylinder");
      break;
    case XP_SRC_EXPLICIT:
      if (!src->positions || !src->directions || !src->polarizations)
        return fail(ctx, XP_ERR_INVALID_ARG, "EXPLICIT needs positions, directions, polarizations");
      break;
    default:
      return fail(ctx, XP_ERR_INVALID_ARG, "unknown source kind");
  }
  if (!(src->wavelength_nm >= 0.0f) || !std::isfinite(src->wavelength_nm) ||
      !(src->wavelength_fwhm_nm >= 0.0f) || !std::isfinite(src->wavelength_fwhm_nm))
    return fail(ctx, XP_ERR_INVALID_ARG, "wavelength and FWHM must be finite and >= 0");
  for (const xp_surface& sf : ctx->surfs)
    if (sf.model == XP_SURF_THIN_FILM && !(src->wavelength_nm > 0.0f))
      return fail(ctx, XP_ERR_INVALID_ARG, "a thin-film surface needs a wavelength > 0");
  if (src->time_profile == XP_TIME_SCINTILLATION) {
    if (!finite_pos(src->tau_singlet_ns) || !finite_pos(src->tau_triplet_ns) ||
        !(src->singlet_fraction >= 0.0f && src->singlet_fraction <= 1.0f))
      return fail(ctx, XP_ERR_INVALID_ARG,
                  "scintillation profile needs decay constants > 0 and a singlet fraction in [0, 1]");
  } else if (src->time_profile != XP_TIME_ZERO) {
    return fail(ctx, XP_ERR_INVALID_ARG, "unknown time profile");
  }
  lc = lc_in ? *lc_in : (ctx->tuned ? ctx->tuned_cfg : default_cfg());
  if (lc.block_size == 0) lc.block_size = 256;
  if (lc.chunk <= 0) lc.chunk = 64;
  // lds_levels < 0: automatic (four staged levels, three where the fourth
  // would lower the occupancy or leave the launch's LDS tallies no room); the
  // resolved configuration keeps -1 so that choose_block_tally may still drop
  // the fourth level
  const bool auto_levels = lc.lds_levels < 0;
  if (auto_levels) lc.lds_levels = -1;
  if (lc.stack_lds == 0) lc.stack_lds = xp::kStackLds;
  if (lc.wave_batch == 0) lc.wave_batch = xp::kWaveBatch;
  if (lc.wave_batch < 1 || lc.wave_batch > 64)
    return fail(ctx, XP_ERR_INVALID_ARG, "wave_batch must be in 1..64");
  if (lc.block_tally < -1 || lc.block_tally > 1)
    return fail(ctx, XP_ERR_INVALID_ARG, "block_tally must be -1, 0 or 1");
  if (lc.stack_lds < 4 || lc.stack_lds > 64 || (lc.stack_lds & (lc.stack_lds - 1)))
    return fail(ctx, XP_ERR_INVALID_ARG, "stack_lds must be a power of two in 4..64");
  if (lc.block_size != 64 && lc.block_size != 128 && lc.block_size != 256)
    return fail(ctx, XP_ERR_INVALID_ARG, "block_size must be 64, 128 or 256");
  if (lc.lds_levels > 4) return fail(ctx, XP_ERR_INVALID_ARG, "lds_levels must be <= 4");
  if (lc.chunk > (1 << 20)) return fail(ctx, XP_ERR_INVALID_ARG, "chunk too large");

  std::memset(&a, 0, sizeof(a));
  a.nodes = ctx->d_nodes;
  a.tris = ctx->d_tris;
  a.n_tris = int32_t(ctx->stats.n_references);
  a.channel_of_sensor = ctx->d_channel;
  const int levels = std::min<int>(auto_levels ? 4 : lc.lds_levels, int(ctx->bvh.level_end.size()));
  a.n_lds_nodes = levels > 0 ? ctx->bvh.level_end[levels - 1] : 0;
  a.stack_lds = lc.stack_lds;
  a.stack_total = ctx->bvh.max_stack;
  a.stack_overflow = ctx->d_stack_overflow;
  a.n_channels = ctx->n_channels;
  a.n_sensors = ctx->max_sensor + 1;
  a.src_kind = src->kind;
  a.medium = src->medium;
  a.n_photons = src->n_photons;
  a.n_sources = src->n_sources;
  a.positions = src->positions;
  a.offsets = src->kind == XP_SRC_POINTS ? src->offsets : nullptr;
  a.count_per_source = src->count_per_source;
  a.per_source_events = src->kind == XP_SRC_POINTS ? src->per_source_events : 0;
  a.chunk = lc.chunk;
  a.wave_batch = lc.wave_batch;
  a.dirs = src->directions;
  a.pols = src->polarizations;
  a.cyl_r = src->cyl_radius;
  a.cyl_zlo = src->cyl_zlo;
  a.cyl_zhi = src->cyl_zhi;
  a.wl_mean = src->wavelength_nm;
  a.wl_sigma = float(double(src->wavelength_fwhm_nm) / (2.0 * std::sqrt(2.0 * std::log(2.0))));
  a.time_profile = src->time_profile;
  a.tau_singlet = src->tau_singlet_ns;
  a.tau_triplet = src->tau_triplet_ns;
  a.singlet_fraction = src->singlet_fraction;
  a.seed_lo = uint32_t(rp->seed);
  a.seed_hi = uint32_t(rp->seed >> 32);
  a.pid_base = rp->pid_base;
  a.max_steps = rp->max_steps > 0 ? rp->max_steps : 10000;
  a.eps = rp->eps;
  a.grad_material = rp->grad_material;
  a.surface_offset = rp->surface_offset;
  for (size_t i = 0; i < ctx->mats.size(); ++i) {
    a.mats[i].n = ctx->mats[i].n;
    a.mats[i].abs_len = ctx->mats[i].abs_length;
    a.mats[i].ray_len = ctx->mats[i].rayleigh_length;
    const auto& t = ctx->disp[i];
    a.disp[i].n = int32_t(t.size());
    for (size_t k = 0; k < t.size(); ++k) {
      a.disp[i].lambda[k] = t[k][0];
      a.disp[i].index[k] = t[k][1];
      a.disp[i].inv_abs[k] = std::isinf(t[k][2]) ? 0.0f : float(1.0 / double(t[k][2]));
      a.disp[i].inv_ray[k] = std::isinf(t[k][3]) ? 0.0f : float(1.0 / double(t[k][3]));
    }
    if (!t.empty()) a.dispersive |= 1 << i;
  }

  for (size_t i = 0; i < ctx->surfs.size(); ++i) {
    const xp_surface& s = ctx->surfs[i];
    // cumulative thresholds of the partition, accumulated in double and rounded once
    const double c1 = double(s.p_detect);
    const double c2 = c1 + s.p_absorb;
    const double c3 = c2 + s.r_diffuse;
    const double c4 = c3 + s.r_specular;
    a.surfs[i].c_detect = float(c1);
    a.surfs[i].c_absorb = float(c2);
    a.surfs[i].c_diffuse = float(c3);
    a.surfs[i].c_specular = float(c4);
    a.surfs[i].p_transmit = s.p_transmit;
    const double rtot = double(s.r_diffuse) + s.r_specular;
    a.surfs[i].inv_r = rtot > 0 ? float(1.0 / rtot) : 0.0f;
    a.surfs[i].inv_t = s.p_transmit > 0 ? float(1.0 / double(s.p_transmit)) : 0.0f;
    a.surfs[i].flags_grad = (s.flags & 0xff) | ((s.grad_param + 1) << 8);
    a.surfs[i].model = s.model;
    a.surfs[i].n_re = s.n_re;
    a.surfs[i].n_im = s.n_im;
    a.surfs[i].film_n = s.film_n;
    a.surfs[i].two_pi_d = float(2.0 * 3.14159265358979323846 * double(s.film_thickness_nm));
  }
  size_t lds = xp::propagate_lds_bytes(a.n_lds_nodes, a.stack_lds, lc.block_size, 0);
  int per_cu = 0;
  hipError_t e = hipSuccess;
  if (lds <= ctx->max_lds) e = xp::max_blocks_per_cu(lc.block_size, lds, false, false, &per_cu);
  if (e != hipSuccess) return hip_fail(ctx, e, "occupancy query");
  if (auto_levels && levels > 3) {
    // the fourth level only where it costs no occupancy
    const int32_t n3 = ctx->bvh.level_end[2];
    const size_t lds3 = xp::propagate_lds_bytes(n3, a.stack_lds, lc.block_size, 0);
    int per_cu3 = 0;
    if (lds3 <= ctx->max_lds) e = xp::max_blocks_per_cu(lc.block_size, lds3, false, false, &per_cu3);
    if (e != hipSuccess) return hip_fail(ctx, e, "occupancy query");
    if (lds > ctx->max_lds || per_cu3 > per_cu) {
      a.n_lds_nodes = n3;
      lds = lds3;
      per_cu = per_cu3;
    }
  }
  if (lds > ctx->max_lds)
    return fail(ctx, XP_ERR_UNSUPPORTED, "LDS request of " + std::to_string(lds) +
                                             " bytes exceeds the device limit; use fewer lds_levels "
                                             "or a smaller block");
  if (per_cu <= 0) return fail(ctx, XP_ERR_UNSUPPORTED, "kernel does not fit on a CU");
  if (lc.blocks_per_cu <= 0 || lc.blocks_per_cu > per_cu) lc.blocks_per_cu = per_cu;
  grid = ctx->n_cu * lc.blocks_per_cu;
  if (int64_t(grid) * lc.block_size > ctx->stack_overflow_lanes)
    return fail(ctx, XP_ERR_UNSUPPORTED, "launch exceeds the traversal-stack overflow area");
  return XP_OK;
}

// Per-wave event caches of a forward launch with per-event hit maps, prefix
// offsets and at most 64 channels, whose map is too large for the LDS block
// tally: each wave sums the hit-map rows of its two most recent events in LDS
// and adds them to device memory when it moves on, instead of one
// device-memory atomic per detected photon.  Only where the extra LDS costs
// no occupancy.  The first 90 % of the photon ids then go out in chunks of
// kBigChunk ids (a wave meets many photons of one event), the rest in the
// launch's chunks (an even end).
void choose_event_cache(const xp_context* ctx, const xp_launch_cfg& cfg, bool records_or_stats,
                        xp::LaunchArgs& a) {
  a.event_cache = 0;
  a.n_big_chunks = 0;
  if (!(a.src_kind == XP_SRC_POINTS && a.offsets && a.per_source_events && a.hit_map) ||
      records_or_stats || a.tally_bytes > 0 || ctx->n_channels > 64)
    return;
  const size_t lds = xp::propagate_lds_bytes(a.n_lds_nodes, a.stack_lds, cfg.block_size, 0) +
                     xp::event_cache_lds_bytes(cfg.block_size);
  int per_cu = 0;
  if (lds > ctx->max_lds ||
      xp::max_blocks_per_cu(cfg.block_size, lds, false, false, &per_cu) != hipSuccess ||
      per_cu < cfg.blocks_per_cu)
    return;
  a.event_cache = 1;
  a.n_big_chunks = int64_t(0.9 * double(a.n_photons)) / xp::kBigChunk;
}

// Choose the per-workgroup LDS tallies of a forward launch: they remove the
// atomic contention of tables whose few cells are hit by photons from every
// workgroup at once: small hit maps (every detection of a short-path
// detector), the loss table (every photon's end) and the arrival-time
// histogram (every detection).  The hit map goes to LDS for at most
// kAutoTallyCells cells (any size that fits with block_tally 1), the other
// two whenever they fit.  Launches with records or counters, block_tally -1,
// or tallies that would lower the occupancy keep the device-memory atomics.
// Expects a.time_hist / a.loss and their sizes to be set.
void choose_block_tally(const xp_context* ctx, const xp_sources* src, const xp_launch_cfg& cfg,
                        bool hits, bool grad, bool records, bool count, xp::LaunchArgs& a) {
  a.tally_cells = 0;
  a.tally_bytes = 0;
  a.lds_time_off = a.lds_loss_off = -1;
  a.n_time_cells = a.n_loss_cells = 0;
  if (cfg.block_tally < 0 || records || count) return;
  const int64_t n_events =
      (src->kind == XP_SRC_POINTS && src->per_source_events) ? src->n_sources : 1;
  size_t bytes = 0;
  const int64_t cells = n_events * int64_t(ctx->n_channels);
  if ((hits || grad) && cells > 0 &&
      cells <= (cfg.block_tally > 0 ? int64_t(1) << 20 : xp::kAutoTallyCells)) {
    const size_t b = xp::tally_lds_bytes(int32_t(cells), grad);
    if (b <= xp::kMaxTallyBytes) {
      a.tally_cells = int32_t(cells);
      bytes = b;
    }
  }
  if (a.loss) {
    const int64_t n = (int64_t(a.n_groups) + int64_t(ctx->mats.size())) * 8;
    if (size_t(n) * 8 <= xp::kMaxLossTallyBytes) {
      a.lds_loss_off = int32_t(bytes);
      a.n_loss_cells = int32_t(n);
      bytes += (size_t(n) * 8 + 15) & ~size_t(15);
    }
  }
  if (a.time_hist) {
    const int64_t n = n_events * int64_t(a.n_time_bins);
    if (size_t(n) * 4 <= xp::kMaxTimeTallyBytes) {
      a.lds_time_off = int32_t(bytes);
      a.n_time_cells = int32_t(n);
      bytes += (size_t(n) * 4 + 15) & ~size_t(15);
    }
  }
  if (bytes == 0) return;
  bytes = (bytes + 127) & ~size_t(127);  // the staged nodes after them stay 128-byte aligned
  auto fits = [&](int32_t n_nodes) {
    const size_t lds = xp::propagate_lds_bytes(n_nodes, a.stack_lds, cfg.block_size, bytes);
    int per_cu = 0;
    return lds <= ctx->max_lds &&
           xp::max_blocks_per_cu(cfg.block_size, lds, false, true, &per_cu) == hipSuccess &&
           per_cu >= cfg.blocks_per_cu;
  };
  if (fits(a.n_lds_nodes)) {
    a.tally_bytes = int32_t(bytes);
    return;
  }
  // automatic levels: the tallies take the fourth staged level's LDS
  if (cfg.lds_levels < 0 && ctx->bvh.level_end.size() >= 4 &&
      a.n_lds_nodes > ctx->bvh.level_end[2] && fits(ctx->bvh.level_end[2])) {
    a.n_lds_nodes = ctx->bvh.level_end[2];
    a.tally_bytes = int32_t(bytes);
    return;
  }
  a.tally_cells = 0;  // does not fit: every table to device memory
  a.lds_time_off = a.lds_loss_off = -1;
  a.n_time_cells = a.n_loss_cells = 0;
}

// fixed_counter: the work counter to use (the fixed scratch's), else one of
// the context's
int launch(xp_context* ctx, xp::LaunchArgs& a, int mode, bool grad, bool records, bool count,
           const xp_launch_cfg& lc, int grid, hipStream_t s,
           unsigned long long* fixed_counter = nullptr) {
  if (a.n_photons == 0) return XP_OK;
  // A launch captured in a graph keeps its counter for every replay, so it
  // gets one that no other launch will use; eager launches reuse the ring.
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(s, &cap);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamIsCapturing");
  unsigned long long* counter;
  if (fixed_counter != nullptr) {
    counter = fixed_counter;
  } else if (cap == hipStreamCaptureStatusActive) {
    if (ctx->graph_next >= xp::kGraphCounters)
      return fail(ctx, XP_ERR_UNSUPPORTED, "more than " + std::to_string(xp::kGraphCounters) +
                                               " launches captured in graphs on this context");
    counter = ctx->d_graph_counters + ctx->graph_next++;
  } else {
    counter = ctx->d_counters + (ctx->ring_next++ % xp::kCounterRing);
  }
  a.work_counter = counter;
  e = xp::launch_reset(counter, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "launch(reset)");
  e = xp::launch_propagate(a, mode, grad, records, count, lc.block_size, grid, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "launch(propagate)");
  return XP_OK;
}

}  // namespace

extern "C" {

const char* xp_version(void) { return "xephot 0.1 (gfx950)"; }

const char* xp_last_error(const xp_context* ctx) {
  return ctx ? ctx->err.c_str() : g_thread_err.c_str();
}

int xp_context_create(int hip_device, xp_context** out) {
  try {
    if (!out) return fail(nullptr, XP_ERR_INVALID_ARG, "null output pointer");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDeviceCount");
    if (hip_device < 0 || hip_device >= n)
      return fail(nullptr, XP_ERR_INVALID_ARG, "no such HIP device");
    DeviceGuard g(hip_device);
    if (g.status != hipSuccess) return hip_fail(nullptr, g.status, "hipSetDevice");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, hip_device);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDeviceProperties");
    xp_context* ctx = new xp_context();
    ctx->device = hip_device;
    ctx->n_cu = prop.multiProcessorCount;
    ctx->max_lds = prop.sharedMemPerBlock;
    e = xp::scratch_init(hip_device);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetSymbolAddress(scratch)");
    e = hipMalloc(&ctx->d_counters,
                  (xp::kCounterRing + xp::kGraphCounters) * sizeof(unsigned long long));
    if (e != hipSuccess) {
      delete ctx;
      return hip_fail(nullptr, e, "hipMalloc(work counters)");
    }
    ctx->d_graph_counters = ctx->d_counters + xp::kCounterRing;
    *out = ctx;
    return XP_OK;
  } catch (const std::bad_alloc&) {
    return fail(nullptr, XP_ERR_OOM, "host allocation failed");
  } catch (...) {
    return fail(nullptr, XP_ERR_HIP, "unexpected exception");
  }
}

void xp_context_destroy(xp_context* ctx) {
  if (!ctx) return;
  DeviceGuard g(ctx->device);
  dfree(ctx->d_nodes);
  dfree(ctx->d_tris);
  dfree(ctx->d_channel);
  dfree(ctx->d_tri_group);
  dfree(ctx->d_counters);
  dfree(ctx->d_stack_overflow);
  delete ctx;
}

// The geometric checks of a mesh: sizes, finite coordinates, vertex indices
// in range, no degenerate triangle.
int check_geometry(xp_context* ctx, const float* vtx, int64_t nv, const int32_t* tri, int64_t nt) {
  if (nv <= 0 || nt <= 0 || nt >= (int64_t(1) << 31) || nv >= (int64_t(1) << 31))
    return fail(ctx, XP_ERR_INVALID_ARG, "nv and nt must be in [1, 2^31)");
  for (int64_t i = 0; i < 3 * nv; ++i)
    if (!std::isfinite(vtx[i]))
      return fail(ctx, XP_ERR_MESH, "non-finite vertex coordinate at vertex " + std::to_string(i / 3));
  for (int64_t t = 0; t < nt; ++t) {
    const int32_t* q = tri + 3 * t;
    for (int k = 0; k < 3; ++k)
      if (q[k] < 0 || q[k] >= nv)
        return fail(ctx, XP_ERR_MESH, "triangle " + std::to_string(t) + " has a vertex index out of range");
    const float* p0 = vtx + 3 * int64_t(q[0]);
    const float* p1 = vtx + 3 * int64_t(q[1]);
    const float* p2 = vtx + 3 * int64_t(q[2]);
    const double e1[3] = {double(p1[0]) - p0[0], double(p1[1]) - p0[1], double(p1[2]) - p0[2]};
    const double e2[3] = {double(p2[0]) - p0[0], double(p2[1]) - p0[1], double(p2[2]) - p0[2]};
    const double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
                 cz = e1[0] * e2[1] - e1[1] * e2[0];
    if (0.5 * std::sqrt(cx * cx + cy * cy + cz * cz) < 1e-12)
      return fail(ctx, XP_ERR_MESH, "triangle " + std::to_string(t) + " is degenerate (area < 1e-12 m^2)");
  }
  return XP_OK;
}

// BVH build options with their defaults filled in (the split budget's
// default depends on the triangle count nt).
int parse_bvh_options(xp_context* ctx, const xp_bvh_options* opts, int64_t nt, int& leaf,
                      int& bins, double& split_budget) {
  leaf = opts && opts->max_leaf_size ? opts->max_leaf_size : 1;
  bins = opts && opts->sah_bins ? opts->sah_bins : 32;
  const float sb = opts ? opts->split_budget : 0.0f;
  if (!(sb <= 4.0f)) return fail(ctx, XP_ERR_INVALID_ARG, "split_budget must be at most 4");
  split_budget = sb == 0.0f ? xp::default_split_budget(nt) : (sb < 0.0f ? 0.0 : double(sb));
  if (leaf < 1 || leaf > 8 || bins < 4 || bins > 64)
    return fail(ctx, XP_ERR_INVALID_ARG, "max_leaf_size must be 1..8, sah_bins 4..64");
  return XP_OK;
}

int xp_load_mesh(xp_context* ctx, const float* vtx, int64_t nv, const int32_t* tri, int64_t nt,
                 const int32_t* mat_inner, const int32_t* mat_outer, const int32_t* surface,
                 const int32_t* sensor) {
  if (!ctx) return fail(nullptr, XP_ERR_INVALID_ARG, "null context");
  try {
    if (!vtx || !tri || !mat_inner || !mat_outer || !surface || !sensor)
      return fail(ctx, XP_ERR_INVALID_ARG, "null mesh array");
    const int gc = check_geometry(ctx, vtx, nv, tri, nt);
    if (gc != XP_OK) return gc;
    int32_t mm = -1, ms = -1, mse = -1;
    for (int64_t t = 0; t < nt; ++t) {
      if (mat_inner[t] < 0 || mat_inner[t] > 255 || mat_outer[t] < 0 || mat_outer[t] > 255)
        return fail(ctx, XP_ERR_MESH, "triangle " + std::to_string(t) + " has a material id outside [0, 255]");
      if (surface[t] < -1 || surface[t] > 65534)
        return fail(ctx, XP_ERR_MESH, "triangle " + std::to_string(t) + " has a surface id outside [-1, 65534]");
      if (sensor[t] < -1)
        return fail(ctx, XP_ERR_MESH, "triangle " + std::to_string(t) + " has a sensor id < -1");
      mm = std::max(mm, std::max(mat_inner[t], mat_outer[t]));
      ms = std::max(ms, surface[t]);
      mse = std::max(mse, sensor[t]);
    }
    ctx->vtx.assign(vtx, vtx + 3 * nv);
    ctx->tri.assign(tri, tri + 3 * nt);
    ctx->mat_in.assign(mat_inner, mat_inner + nt);
    ctx->mat_out.assign(mat_outer, mat_outer + nt);
    ctx->surf.assign(surface, surface + nt);
    ctx->sensor.assign(sensor, sensor + nt);
    ctx->max_mat = mm;
    ctx->max_surf = ms;
    ctx->max_sensor = mse;
    ctx->mesh_loaded = true;
    ctx->bvh_built = false;
    ctx->tuned = false;
    ctx->n_groups = 0;  // loss groups refer to the previous mesh
    return XP_OK;
  } catch (const std::bad_alloc&) {
    return fail(ctx, XP_ERR_OOM, "host allocation failed");
  } catch (...) {
    return fail(ctx, XP_ERR_HIP, "unexpected exception");
  }
}

int xp_set_materials(xp_context* ctx, const xp_material* m, int32_t n) {
  if (!ctx) return fail(nullptr, XP_ERR_INVALID_ARG, "null context");
  if (!m || n <= 0 || n > xp::kMaxMaterials)
    return fail(ctx, XP_ERR_INVALID_ARG, "need 1..8 materials");
  for (int32_t i = 0; i < n; ++i) {
    if (!finite_pos(m[i].n)) return fail(ctx, XP_ERR_INVALID_ARG, "refractive index must be finite and > 0");
    if (!(m[i].abs_length > 0.0f) || !(m[i].rayleigh_length > 0.0f))
      return fail(ctx, XP_ERR_INVALID_ARG, "lengths must be > 0 (INFINITY allowed)");
  }
  try {
    ctx->mats.assign(m, m + n);
    ctx->disp.assign(size_t(n), {});
  } catch (...) {
    return fail(ctx, XP_ERR_OOM, "host allocation failed");
  }
  return XP_OK;
}

int xp_set_material_dispersion(xp_context* ctx, int32_t material, int32_t n_points,
                               const float* lambda_nm, const float* index,
                               const float* abs_length, const float* rayleigh_length) {
  if (!ctx) return fail(nullptr, XP_ERR_INVALID_ARG, "null context");
  if (material < 0 || material >= int32_t(ctx->mats.size()))
    return fail(ctx, XP_ERR_STATE, "material id not in the material table");
  if (n_points < 0 || n_points > xp::kMaxDispersion)
    return fail(ctx, XP_ERR_INVALID_ARG, "a dispersion table has 0..8 samples");
  if (n_points > 0 && (!lambda_nm || !index || !abs_length || !rayleigh_length))
    return fail(ctx, XP_ERR_INVALID_ARG, "null dispersion array");
  for (int32_t i = 0; i < n_points; ++i) {
    if (!finite_pos(lambda_nm[i]) || (i > 0 && !(lambda_nm[i] > lambda_nm[i - 1])))
      return fail(ctx, XP_ERR_INVALID_ARG, "wavelengths must be finite, > 0 and ascending");
    if (!finite_pos(index[i]) || !(abs_length[i] > 0.0f) || !(rayleigh_length[i] > 0.0f))
      return fail(ctx, XP_ERR_INVALID_ARG, "index finite > 0, lengths > 0 (INFINITY allowed)");
  }
  try {
    auto& t = ctx->disp[size_t(material)];
    t.clear();
    for (int32_t i = 0; i < n_points; ++i)
      t.push_back({lambda_nm[i], index[i], abs_length[i], rayleigh_length[i]});
  } catch (...) {
    return fail(ctx, XP_ERR_OOM, "host allocation failed");
  }
  return XP_OK;
}

int xp_set_surfaces(xp_context* ctx, const xp_surface* s, int32_t n) {
  if (!ctx) return fail(nullptr, XP_ERR_INVALID_ARG, "null context");
  if (!s || n <= 0 || n > xp::kMaxSurfaces)
    return fail(ctx, XP_ERR_INVALID_ARG, "need 1..16 surfaces");
  for (int32_t i = 0; i < n; ++i) {
    if (s[i].flags & ~XP_SURF_DETECT_FRONT_ONLY)
      return fail(ctx, XP_ERR_INVALID_ARG, "unknown surface flag");
    if (s[i].model == XP_SURF_COMPLEX_INDEX || s[i].model == XP_SURF_THIN_FILM) {
      if (!finite_pos(s[i].n_re) || !(s[i].n_im >= 0.0f) || !std::isfinite(s[i].n_im))
        return fail(ctx, XP_ERR_INVALID_ARG, "surface " + std::to_string(i) + ": complex index needs n_re > 0, n_im >= 0");
      if (s[i].model == XP_SURF_THIN_FILM &&
          (!finite_pos(s[i].film_n) || !(s[i].film_thickness_nm >= 0.0f) ||
           !std::isfinite(s[i].film_thickness_nm)))
        return fail(ctx, XP_ERR_INVALID_ARG, "surface " + std::to_string(i) + ": film needs film_n > 0, thickness >= 0");
      if (s[i].grad_param != -1)
        return fail(ctx, XP_ERR_INVALID_ARG, "surface " + std::to_string(i) + ": reflectance models take no gradient tag");
      continue;
    }
    if (s[i].model != XP_SURF_EXPLICIT)
      return fail(ctx, XP_ERR_INVALID_ARG, "unknown surface model");
    const float p[5] = {s[i].p_detect, s[i].p_absorb, s[i].r_diffuse, s[i].r_specular,
                        s[i].p_transmit};
    double sum = 0.0;
    for (float x : p) {
      if (!(x >= 0.0f && x <= 1.0f))
        return fail(ctx, XP_ERR_INVALID_ARG, "surface " + std::to_string(i) + ": probability outside [0, 1]");
      sum += x;
    }
    if (std::fabs(sum - 1.0) > 1e-6)
      return fail(ctx, XP_ERR_INVALID_ARG, "surface " + std::to_string(i) + ": probabilities do not sum to 1");
    if (s[i].grad_param != -1 && s[i].grad_param != 2 && s[i].grad_param != 3)
      return fail(ctx, XP_ERR_INVALID_ARG, "grad_param must be -1, 2 or 3");
  }
  try {
    ctx->surfs.assign(s, s + n);
  } catch (...) {
    return fail(ctx, XP_ERR_OOM, "host allocation failed");
  }
  return XP_OK;
}

int xp_set_channel_map(xp_context* ctx, const int32_t* channel_of_sensor, int32_t n_sensors,
                       int32_t n_channels) {
  if (!ctx) return fail(nullptr, XP_ERR_INVALID_ARG, "null context");
  if (!channel_of_sensor || n_sensors <= 0 || n_channels <= 0)
    return fail(ctx, XP_ERR_INVALID_ARG, "need a map of n_sensors > 0 entries and n_channels > 0");
  for (int32_t i = 0; i < n_sensors; ++i)
    if (channel_of_sensor[i] < 0 || channel_of_sensor[i] >= n_channels)
      return fail(ctx, XP_ERR_INVALID_ARG, "channel of sensor " + std::to_string(i) + " out of range");
  try {
    ctx->channel.assign(channel_of_sensor, channel_of_sensor + n_sensors);
  } catch (...) {
    return fail(ctx, XP_ERR_OOM, "host allocation failed");
  }
  ctx->n_channels = n_channels;
  ctx->channel_set = true;
  if (ctx->bvh_built) {
    DeviceGuard g(ctx->device);
    if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
    return upload_channel_map(ctx);
  }
  return XP_OK;
}

int xp_build_bvh(xp_context* ctx, const xp_bvh_options* opts) {
  if (!ctx) return fail(nullptr, XP_ERR_INVALID_ARG, "null context");
  if (!ctx->mesh_loaded) return fail(ctx, XP_ERR_STATE, "xp_load_mesh has not been called");
  int leaf = 1, bins = 32;
  double split_budget = 0.0;
  const int oc = parse_bvh_options(ctx, opts, int64_t(ctx->mat_in.size()), leaf, bins, split_budget);
  if (oc != XP_OK) return oc;
  if (int64_t(ctx->mat_in.size()) >= xp::kMaxReferences)
    return fail(ctx, XP_ERR_UNSUPPORTED, "the BVH addresses fewer than 2^24 triangles");
  if (ctx->channel_set && int32_t(ctx->channel.size()) <= ctx->max_sensor)
    return fail(ctx, XP_ERR_STATE, "channel map does not cover the mesh's sensor ids");
  try {
    const auto t0 = std::chrono::steady_clock::now();
    xp::BvhResult r;
    std::string err;
    const int64_t nt = int64_t(ctx->mat_in.size());
    if (!xp::build_bvh4(ctx->vtx.data(), ctx->tri.data(), nt, ctx->mat_in.data(),
                        ctx->mat_out.data(), ctx->surf.data(), ctx->sensor.data(), leaf, bins,
                        split_budget, r, err))
      return fail(ctx, XP_ERR_MESH, err);
    if (r.max_stack > 512) return fail(ctx, XP_ERR_UNSUPPORTED, "BVH too deep");
    DeviceGuard g(ctx->device);
    if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
    ctx->bvh_built = false;
    ctx->tuned = false;
    dfree(ctx->d_nodes);
    dfree(ctx->d_tris);
    hipError_t e = hipMalloc(&ctx->d_nodes, r.nodes.size() * sizeof(xp::Node4));
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMalloc(nodes)");
    e = hipMalloc(&ctx->d_tris, r.tris.size() * sizeof(xp::TriRec));
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMalloc(triangles)");
    e = hipMemcpy(ctx->d_nodes, r.nodes.data(), r.nodes.size() * sizeof(xp::Node4), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpy(nodes)");
    e = hipMemcpy(ctx->d_tris, r.tris.data(), r.tris.size() * sizeof(xp::TriRec), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpy(triangles)");
    // spill slots for every lane that can be resident at once (allocated here,
    // never inside a launch, so that launches can be captured in a graph)
    dfree(ctx->d_stack_overflow);
    ctx->stack_overflow_lanes = int64_t(ctx->n_cu) * xp::kMaxThreadsPerCu;
    e = hipMalloc(&ctx->d_stack_overflow,
                  size_t(ctx->stack_overflow_lanes) * size_t(r.max_stack) * sizeof(int32_t));
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMalloc(stack overflow)");
    const int rc = upload_channel_map(ctx);
    if (rc != XP_OK) return rc;
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    ctx->stats.n_nodes = int64_t(r.nodes.size());
    ctx->stats.n_triangles = nt;
    ctx->stats.n_references = r.n_refs;
    ctx->stats.depth = r.depth;
    ctx->stats.max_stack = r.max_stack;
    ctx->stats.node_bytes = int64_t(r.nodes.size() * sizeof(xp::Node4));
    ctx->stats.triangle_bytes = int64_t(r.tris.size() * sizeof(xp::TriRec));
    ctx->stats.build_seconds = secs;
    r.nodes.clear();
    r.nodes.shrink_to_fit();
    r.tris.clear();
    r.tris.shrink_to_fit();
    ctx->bvh = std::move(r);
    ctx->bvh_built = true;
    return XP_OK;
  } catch (const std::bad_alloc&) {
    return fail(ctx, XP_ERR_OOM, "host allocation failed");
  } catch (...) {
    return fail(ctx, XP_ERR_HIP, "unexpected exception");
  }
}

int xp_bvh_build_host(const float* vtx, int64_t nv, const int32_t* tri, int64_t nt,
                      const xp_bvh_options* opts, xp_bvh_info* info, void* nodes,
                      int64_t nodes_capacity, void* records, int64_t records_capacity) {
  if (!vtx || !tri || !info) return fail(nullptr, XP_ERR_INVALID_ARG, "null argument");
  try {
    if (nt >= xp::kMaxReferences)
      return fail(nullptr, XP_ERR_UNSUPPORTED, "the BVH addresses fewer than 2^24 triangles");
    int rc = check_geometry(nullptr, vtx, nv, tri, nt);
    if (rc != XP_OK) return rc;
    int leaf = 1, bins = 32;
    double split_budget = 0.0;
    rc = parse_bvh_options(nullptr, opts, nt, leaf, bins, split_budget);
    if (rc != XP_OK) return rc;
    const auto t0 = std::chrono::steady_clock::now();
    const std::vector<int32_t> zero(size_t(nt), 0), none(size_t(nt), -1);
    xp::BvhResult r;
    std::string err;
    if (!xp::build_bvh4(vtx, tri, nt, zero.data(), zero.data(), none.data(), none.data(), leaf,
                        bins, split_budget, r, err))
      return fail(nullptr, XP_ERR_MESH, err);
    *info = xp_bvh_info{};
    info->n_nodes = int64_t(r.nodes.size());
    info->n_triangles = nt;
    info->n_references = r.n_refs;
    info->depth = r.depth;
    info->max_stack = r.max_stack;
    info->node_bytes = int64_t(r.nodes.size() * sizeof(xp::Node4));
    info->triangle_bytes = int64_t(r.tris.size() * sizeof(xp::TriRec));
    info->build_seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (nodes) {
      if (nodes_capacity < info->n_nodes)
        return fail(nullptr, XP_ERR_INVALID_ARG, "node buffer too small");
      std::memcpy(nodes, r.nodes.data(), r.nodes.size() * sizeof(xp::Node4));
    }
    if (records) {
      if (records_capacity < int64_t(r.tris.size()))
        return fail(nullptr, XP_ERR_INVALID_ARG, "record buffer too small");
      std::memcpy(records, r.tris.data(), r.tris.size() * sizeof(xp::TriRec));
    }
    return XP_OK;
  } catch (const std::bad_alloc&) {
    return fail(nullptr, XP_ERR_OOM, "host allocation failed");
  } catch (...) {
    return fail(nullptr, XP_ERR_INVALID_ARG, "unexpected exception");
  }
}

int xp_bvh_stats(const xp_context* ctx, xp_bvh_info* out) {
  if (!ctx || !out) return fail(nullptr, XP_ERR_INVALID_ARG, "null argument");
  if (!ctx->bvh_built) return fail(const_cast<xp_context*>(ctx), XP_ERR_STATE, "no BVH");
  *out = ctx->stats;
  return XP_OK;
}

}  // extern "C"

namespace {

// Forward launch of xp_propagate_ex (use_scratch false: the context's work
// counters and stack overflow area) and of xp_propagate_static (true: the
// fixed device scratch; no allocation, fewer workgroups per CU if the
// overflow area would not fit it).
int propagate_forward(xp_context* ctx, const xp_sources* src, const xp_run_params* rp,
                      int32_t* d_hit_map, double* d_grad, xp_photon_record* d_records,
                      uint64_t* d_stats, const xp_extra_tallies* extra, const xp_launch_cfg* lc,
                      xp_stream stream, bool use_scratch) {
  try {
    xp::LaunchArgs a;
    xp_launch_cfg cfg;
    int grid = 0;
    if (!ctx) return fail(nullptr, XP_ERR_INVALID_ARG, "null context");
    DeviceGuard g(ctx->device);
    if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
    int rc = prepare(ctx, src, rp, lc, a, cfg, grid);
    if (rc != XP_OK) return rc;
    if (d_grad && rp->grad_material >= 0 && ((a.dispersive >> rp->grad_material) & 1))
      return fail(ctx, XP_ERR_UNSUPPORTED, "gradient tallies need a gradient material without a dispersion table");
    a.hit_map = d_hit_map;
    a.grad = d_grad;
    a.records = d_records;
    a.stats = reinterpret_cast<unsigned long long*>(d_stats);
    if (extra && extra->d_time_hist) {
      if (extra->n_time_bins < 1 || !finite_pos(extra->time_bin_ns))
        return fail(ctx, XP_ERR_INVALID_ARG, "time histogram needs n_time_bins >= 1 and a bin width > 0");
      const float inv = float(1.0 / double(extra->time_bin_ns));
      if (!std::isfinite(inv) || !(inv > 0.0f))
        return fail(ctx, XP_ERR_INVALID_ARG, "time bin width out of range");
      a.time_hist = extra->d_time_hist;
      a.n_time_bins = extra->n_time_bins;
      a.time_inv_bin = inv;
    }
    if (extra && extra->d_loss) {
      if (ctx->n_groups <= 0)
        return fail(ctx, XP_ERR_STATE, "loss tally requested but xp_set_loss_groups has not been called");
      a.loss = reinterpret_cast<unsigned long long*>(extra->d_loss);
      a.tri_group = ctx->d_tri_group;
      a.n_groups = ctx->n_groups;
    }
    unsigned long long* fixed_counter = nullptr;
    if (use_scratch) {
      char* base = static_cast<char*>(xp::scratch_base(ctx->device));
      if (base == nullptr) return fail(ctx, XP_ERR_STATE, "device scratch not set up");
      // the overflow area holds stack_total entries per lane of the launch
      const size_t per_lane = size_t(a.stack_total) * sizeof(int32_t);
      const size_t room = xp::kScratchBytes - xp::kScratchCounterBytes;
      const bool caller_fixed = lc != nullptr && lc->blocks_per_cu > 0;
      while (size_t(grid) * size_t(cfg.block_size) * per_lane > room) {
        if (caller_fixed || cfg.blocks_per_cu <= 1)
          return fail(ctx, XP_ERR_UNSUPPORTED,
                      "the launch's traversal-stack overflow area needs " +
                          std::to_string(size_t(grid) * size_t(cfg.block_size) * per_lane) +
                          " bytes; the fixed scratch holds " + std::to_string(room) +
                          " (fewer blocks_per_cu or a smaller block_size)");
        cfg.blocks_per_cu -= 1;
        grid = ctx->n_cu * cfg.blocks_per_cu;
      }
      fixed_counter = reinterpret_cast<unsigned long long*>(base);
      a.stack_overflow = reinterpret_cast<int32_t*>(base + xp::kScratchCounterBytes);
    }
    choose_block_tally(ctx, src, cfg, d_hit_map != nullptr, d_grad != nullptr, d_records != nullptr,
                       d_stats != nullptr, a);
    choose_event_cache(ctx, cfg, d_records != nullptr || d_stats != nullptr, a);
    return launch(ctx, a, xp::kForward, d_grad != nullptr, d_records != nullptr, d_stats != nullptr,
                  cfg, grid, static_cast<hipStream_t>(stream), fixed_counter);
  } catch (...) {
    return fail(ctx, XP_ERR_HIP, "unexpected exception");
  }
}

}  // namespace

extern "C" {

int xp_propagate_ex(xp_context* ctx, const xp_sources* src, const xp_run_params* rp,
                    int32_t* d_hit_map, double* d_grad, xp_photon_record* d_records,
                    uint64_t* d_stats, const xp_extra_tallies* extra, const xp_launch_cfg* lc,
                    xp_stream stream) {
  return propagate_forward(ctx, src, rp, d_hit_map, d_grad, d_records, d_stats, extra, lc, stream,
                           false);
}

int xp_propagate_static(xp_context* ctx, const xp_sources* src, const xp_run_params* rp,
                        int32_t* d_hit_map, double* d_grad, xp_photon_record* d_records,
                        uint64_t* d_stats, const xp_launch_cfg* lc, xp_stream stream) {
  return propagate_forward(ctx, src, rp, d_hit_map, d_grad, d_records, d_stats, nullptr, lc,
                           stream, true);
}

int xp_propagate(xp_context* ctx, const xp_sources* src, const xp_run_params* rp, int32_t* d_hit_map,
                 double* d_grad, xp_photon_record* d_records, uint64_t* d_stats,
                 const xp_launch_cfg* lc, xp_stream stream) {
  return xp_propagate_ex(ctx, src, rp, d_hit_map, d_grad, d_records, d_stats, nullptr, lc, stream);
}

int xp_set_loss_groups(xp_context* ctx, const int32_t* group_of_triangle, int32_t n_groups) {
  if (!ctx) return fail(nullptr, XP_ERR_INVALID_ARG, "null context");
  if (!ctx->mesh_loaded) return fail(ctx, XP_ERR_STATE, "xp_load_mesh has not been called");
  if (!group_of_triangle || n_groups <= 0)
    return fail(ctx, XP_ERR_INVALID_ARG, "need a group per triangle and n_groups > 0");
  const int64_t nt = int64_t(ctx->mat_in.size());
  for (int64_t t = 0; t < nt; ++t)
    if (group_of_triangle[t] < 0 || group_of_triangle[t] >= n_groups)
      return fail(ctx, XP_ERR_INVALID_ARG, "group of triangle " + std::to_string(t) + " out of range");
  try {
    DeviceGuard g(ctx->device);
    if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
    dfree(ctx->d_tri_group);
    ctx->n_groups = 0;
    hipError_t e = hipMalloc(&ctx->d_tri_group, size_t(nt) * sizeof(int32_t));
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMalloc(loss groups)");
    e = hipMemcpy(ctx->d_tri_group, group_of_triangle, size_t(nt) * sizeof(int32_t),
                  hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpy(loss groups)");
    ctx->n_groups = n_groups;
    return XP_OK;
  } catch (...) {
    return fail(ctx, XP_ERR_HIP, "unexpected exception");
  }
}

int xp_time_quantile(const int32_t* d_time_hist, int64_t n_events, int32_t n_time_bins,
                     float time_bin_ns, float q, float* d_out, xp_stream stream) {
  if (n_events < 0 || (n_events > 0 && (!d_time_hist || !d_out)) || n_time_bins < 1 ||
      !finite_pos(time_bin_ns) || !(q > 0.0f && q <= 1.0f))
    return fail(nullptr, XP_ERR_INVALID_ARG,
                "need histograms, n_time_bins >= 1, a bin width > 0 and 0 < q <= 1");
  if (n_events == 0) return XP_OK;
  const hipError_t e = xp::launch_time_quantile(d_time_hist, n_events, n_time_bins, time_bin_ns, q,
                                                d_out, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(nullptr, e, "launch(time_quantile)");
  return XP_OK;
}

int xp_stream_read(const void* buf, int64_t n_vec, int32_t passes, int32_t blocks, float* out,
                   xp_stream stream) {
  if (!buf || !out || n_vec <= 0 || passes <= 0 || blocks <= 0 || blocks > (1 << 20))
    return fail(nullptr, XP_ERR_INVALID_ARG, "bad stream-read arguments");
  const hipError_t e = xp::launch_stream_read(buf, n_vec, passes, blocks, out,
                                              static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(nullptr, e, "launch(stream_read)");
  return XP_OK;
}

int xp_valu_probe(int32_t kind, int32_t iters, int32_t blocks, float* out, xp_stream stream) {
  if (kind < 0 || kind > 5 || iters <= 0 || blocks <= 0 || blocks > (1 << 20) || !out)
    return fail(nullptr, XP_ERR_INVALID_ARG, "bad VALU-probe arguments");
  const hipError_t e = xp::launch_valu_probe(kind, 0.999999f, 1e-7f, iters, blocks, out,
                                             static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(nullptr, e, "launch(valu_probe)");
  return XP_OK;
}

int xp_sample_wavelength(uint64_t seed, uint64_t pid0, int64_t n, float mean_nm, float fwhm_nm,
                         float* out, xp_stream stream) {
  if (n < 0 || (n > 0 && !out) || !(mean_nm >= 0.0f) || !std::isfinite(mean_nm) ||
      !(fwhm_nm >= 0.0f) || !std::isfinite(fwhm_nm))
    return fail(nullptr, XP_ERR_INVALID_ARG, "bad wavelength sampler arguments");
  if (n >= (int64_t(1) << 37)) return fail(nullptr, XP_ERR_INVALID_ARG, "too many samples");
  if (n == 0) return XP_OK;
  const float sigma = float(double(fwhm_nm) / (2.0 * std::sqrt(2.0 * std::log(2.0))));
  const hipError_t e = xp::launch_wavelength(seed, pid0, n, mean_nm, sigma, out,
                                             static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(nullptr, e, "launch(wavelength)");
  return XP_OK;
}

int xp_surface_reflectance(int32_t model, float n1, float n_re, float n_im, float film_n,
                           float film_thickness_nm, float lambda_nm, int64_t n,
                           const float* cos_i, float* out_rs, float* out_rp, xp_stream stream) {
  if ((model != XP_SURF_COMPLEX_INDEX && model != XP_SURF_THIN_FILM) || !finite_pos(n1) ||
      !finite_pos(n_re) || !(n_im >= 0.0f) || !std::isfinite(n_im) ||
      (model == XP_SURF_THIN_FILM && (!finite_pos(film_n) || !(film_thickness_nm >= 0.0f) ||
                                      !finite_pos(lambda_nm))) ||
      n < 0 || (n > 0 && (!cos_i || !out_rs || !out_rp)))
    return fail(nullptr, XP_ERR_INVALID_ARG, "bad reflectance arguments");
  if (n >= (int64_t(1) << 37)) return fail(nullptr, XP_ERR_INVALID_ARG, "too many samples");
  if (n == 0) return XP_OK;
  const float two_pi_d = float(2.0 * 3.14159265358979323846 * double(film_thickness_nm));
  const hipError_t e = xp::launch_reflectance(model, n1, n_re, n_im, film_n, two_pi_d, lambda_nm,
                                              n, cos_i, out_rs, out_rp,
                                              static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(nullptr, e, "launch(reflectance)");
  return XP_OK;
}

int xp_sample_emission_time(uint64_t seed, uint64_t pid0, int64_t n, float tau_singlet_ns,
                            float tau_triplet_ns, float singlet_fraction, float* out_t,
                            int32_t* out_singlet, xp_stream stream) {
  if (n < 0 || (n > 0 && !out_t) || !finite_pos(tau_singlet_ns) || !finite_pos(tau_triplet_ns) ||
      !(singlet_fraction >= 0.0f && singlet_fraction <= 1.0f))
    return fail(nullptr, XP_ERR_INVALID_ARG, "bad emission-time sampler arguments");
  if (n >= (int64_t(1) << 37)) return fail(nullptr, XP_ERR_INVALID_ARG, "too many samples");
  if (n == 0) return XP_OK;
  const hipError_t e = xp::launch_emission_time(seed, pid0, n, tau_singlet_ns, tau_triplet_ns,
                                                singlet_fraction, out_t, out_singlet,
                                                static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(nullptr, e, "launch(emission_time)");
  return XP_OK;
}

int xp_backward(xp_context* ctx, const xp_sources* src, const xp_run_params* rp,
                const float* d_grad_hits, double* d_grad_params, const xp_launch_cfg* lc,
                xp_stream stream) {
  try {
    xp::LaunchArgs a;
    xp_launch_cfg cfg;
    int grid = 0;
    if (!ctx) return fail(nullptr, XP_ERR_INVALID_ARG, "null context");
    if (!d_grad_hits || !d_grad_params)
      return fail(ctx, XP_ERR_INVALID_ARG, "null gradient buffer");
    DeviceGuard g(ctx->device);
    if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
    int rc = prepare(ctx, src, rp, lc, a, cfg, grid);
    if (rc != XP_OK) return rc;
    if (rp->grad_material >= 0 && ((a.dispersive >> rp->grad_material) & 1))
      return fail(ctx, XP_ERR_UNSUPPORTED, "the backward pass needs a gradient material without a dispersion table");
    a.grad_hits = d_grad_hits;
    a.grad_params = d_grad_params;
    return launch(ctx, a, xp::kBackward, false, false, false, cfg, grid,
                  static_cast<hipStream_t>(stream));
  } catch (...) {
    return fail(ctx, XP_ERR_HIP, "unexpected exception");
  }
}

int xp_autotune(xp_context* ctx, const xp_sources* src, const xp_run_params* rp,
                int64_t sample_photons, xp_launch_cfg* out, xp_stream stream) {
  if (!ctx) return fail(nullptr, XP_ERR_INVALID_ARG, "null context");
  if (!src || !rp || sample_photons <= 0) return fail(ctx, XP_ERR_INVALID_ARG, "bad arguments");
  try {
    DeviceGuard g(ctx->device);
    if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
    hipStream_t s = static_cast<hipStream_t>(stream);
    xp_sources sample = *src;
    sample.n_photons = std::min(src->n_photons, sample_photons);
    const int64_t n_events =
        (src->kind == XP_SRC_POINTS && src->per_source_events) ? src->n_sources : 1;
    int32_t* d_map = nullptr;
    const size_t map_bytes = size_t(n_events) * std::max(ctx->n_channels, 1) * sizeof(int32_t);
    hipError_t e = hipMalloc(&d_map, map_bytes);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMalloc(autotune map)");
    hipEvent_t t0, t1;
    (void)hipEventCreate(&t0);
    (void)hipEventCreate(&t1);
    const xp_launch_cfg dflt = default_cfg();
    int rc = XP_OK;
    // best of three timings of one candidate; false if it does not fit the
    // device (skipped) or on an error (rc set)
    auto time_cfg = [&](const xp_launch_cfg& cand, float& ms_out) -> bool {
      xp::LaunchArgs a;
      xp_launch_cfg cfg;
      int grid = 0;
      rc = prepare(ctx, &sample, rp, &cand, a, cfg, grid);
      if (rc == XP_ERR_UNSUPPORTED) {  // does not fit this device: skip the candidate
        rc = XP_OK;
        return false;
      }
      if (rc != XP_OK) return false;
      a.hit_map = d_map;
      choose_block_tally(ctx, &sample, cfg, true, false, false, false, a);
      float ms_best = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        (void)hipEventRecord(t0, s);
        rc = launch(ctx, a, xp::kForward, false, false, false, cfg, grid, s);
        if (rc != XP_OK) return false;
        (void)hipEventRecord(t1, s);
        e = hipEventSynchronize(t1);
        if (e != hipSuccess) {
          rc = hip_fail(ctx, e, "autotune run");
          return false;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, t0, t1);
        ms_best = std::min(ms_best, ms);
      }
      ms_out = ms_best;
      return true;
    };
    float best_ms = 1e30f, default_ms = 1e30f;
    xp_launch_cfg best = dflt;
    auto consider = [&](const xp_launch_cfg& cand) {
      float ms = 0.0f;
      if (!time_cfg(cand, ms)) return;
      if (cand.block_size == dflt.block_size && cand.blocks_per_cu == dflt.blocks_per_cu &&
          cand.chunk == dflt.chunk && cand.lds_levels == dflt.lds_levels &&
          cand.stack_lds == dflt.stack_lds && cand.wave_batch == dflt.wave_batch &&
          cand.block_tally == dflt.block_tally)
        default_ms = ms;
      if (ms < best_ms) {
        best_ms = ms;
        best = cand;
      }
    };
    // stage 1: block size, staged BVH levels, LDS stack window, interaction batch
    for (int b : {64, 256})
      for (int l : {0, -1})
        for (int sl : {8, 16})
          for (int wb : {16, 32, 48}) {
            if (rc == XP_OK) consider(xp_launch_cfg{b, 0, 64, l, sl, wb, 0});
          }
    // stage 2: workgroups per CU below the occupancy limit (0 = the limit),
    // then photon ids per refill, each around the best so far
    const xp_launch_cfg s1 = best;
    for (int bpc : {2, 3, 4}) {
      xp_launch_cfg c = s1;
      c.blocks_per_cu = bpc;
      if (rc == XP_OK) consider(c);
    }
    const xp_launch_cfg s2 = best;
    for (int ch : {16, 32, 128, 256}) {
      xp_launch_cfg c = s2;
      c.chunk = ch;
      if (rc == XP_OK) consider(c);
    }
    // then the best with the block tallies forced on (the default keeps them
    // for small hit maps; the timing runs tally hits only, so it never turns
    // them off for launches that also tally gradients)
    if (rc == XP_OK && best_ms < 1e30f) {
      xp_launch_cfg on = best;
      on.block_tally = 1;
      consider(on);
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    (void)hipFree(d_map);
    if (rc != XP_OK) return rc;
    // the default unless a candidate is clearly faster: timings on a sample
    // of a few milliseconds do not separate configurations within ~2 %
    // (blocks_per_cu 0 is re-derived from the occupancy at launch)
    if (default_ms < 1e30f && best_ms > 0.98f * default_ms) best = dflt;
    ctx->tuned_cfg = best;
    ctx->tuned = true;
    if (out) *out = best;
    return XP_OK;
  } catch (...) {
    return fail(ctx, XP_ERR_HIP, "unexpected exception");
  }
}

int xp_closest_hit(xp_context* ctx, int64_t n, const float* orig, const float* dir,
                   const int32_t* skip, float tmin, float tmax, int32_t brute, int32_t* out_tri,
                   float* out_t, xp_stream stream) {
  if (!ctx) return fail(nullptr, XP_ERR_INVALID_ARG, "null context");
  if (!ctx->bvh_built) return fail(ctx, XP_ERR_STATE, "no BVH");
  if (n < 0 || (n > 0 && (!orig || !dir || !out_tri || !out_t)))
    return fail(ctx, XP_ERR_INVALID_ARG, "bad ray arrays");
  if (n >= (int64_t(1) << 37)) return fail(ctx, XP_ERR_INVALID_ARG, "too many rays");
  DeviceGuard g(ctx->device);
  if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
  int32_t depth_pow2 = 1;
  while (depth_pow2 < ctx->bvh.max_stack + 4) depth_pow2 <<= 1;
  const hipError_t e = xp::launch_closest_hit(
      ctx->d_nodes, ctx->d_tris, int32_t(ctx->stats.n_references), depth_pow2, n, orig, dir,
      skip, tmin, tmax, brute, out_tri, out_t, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(ctx, e, "launch(closest_hit)");
  return XP_OK;
}

int xp_sample(int32_t kind, uint64_t seed, uint64_t pid0, int64_t n, const float* in_dir,
              const float* in_pol, float cyl_radius, float cyl_zlo, float cyl_zhi, float* out_dir,
              float* out_pol, xp_stream stream) {
  if (kind < 0 || kind > 3 || n < 0) return fail(nullptr, XP_ERR_INVALID_ARG, "bad sampler request");
  if (n > 0 && (!out_dir || !out_pol)) return fail(nullptr, XP_ERR_INVALID_ARG, "null output");
  if (n > 0 && (kind == 1 || kind == 2) && !in_dir) return fail(nullptr, XP_ERR_INVALID_ARG, "null input");
  if (n > 0 && kind == 2 && !in_pol) return fail(nullptr, XP_ERR_INVALID_ARG, "null input");
  if (n >= (int64_t(1) << 37)) return fail(nullptr, XP_ERR_INVALID_ARG, "too many samples");
  const hipError_t e = xp::launch_sample(kind, seed, pid0, n, in_dir, in_pol, cyl_radius, cyl_zlo,
                                         cyl_zhi, out_dir, out_pol, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(nullptr, e, "launch(sample)");
  return XP_OK;
}

}  // extern "C"

// xp_internal.h -- data layouts shared by the host side and the gfx950 kernels
// of the photon-transport library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/xephot.h"

namespace xp {

constexpr int kMaxMaterials = 8;
constexpr int kMaxSurfaces = 16;
constexpr int kCounterRing = 64;      // work counters of eager launches, reused in turn
constexpr int kGraphCounters = 256;   // work counters of launches captured in graphs
constexpr int kStatsWords = 24;
constexpr int kStackLds = 16;        // LDS window entries per lane
constexpr int64_t kBigChunk = 768;   // photon ids per chunk of an event-cache launch's first part
constexpr int kEventCacheSlots = 2;  // events whose hit-map rows a wave sums in LDS
// LDS of the event caches: per wave, kEventCacheSlots rows of 64 int32 counters
inline size_t event_cache_lds_bytes(int block) { return size_t(block / 64) * kEventCacheSlots * 64 * 4; }
constexpr int kWaveBatch = 32;       // lanes per wave interaction phase
constexpr int kMaxThreadsPerCu = 2048;
// Default pre-splitting budget: extra BVH references up to 2 % of the
// triangles, but at least 2,048 pieces (at most 4 per triangle).  A mesh of a
// few thousand triangles stays shallow when its fan slivers are split (on a
// 4,128-triangle TPC 0.45-0.6 extra references per triangle are fastest),
// while on a mesh of ~5e5 triangles more than 2 % deepens the tree for little
// gain.
constexpr double kDefaultSplitBudget = 0.02;
constexpr double kDefaultSplitPieces = 2048.0;
inline double default_split_budget(int64_t n_triangles) {
  const double b = n_triangles > 0 ? kDefaultSplitPieces / double(n_triangles) : 4.0;
  return b < kDefaultSplitBudget ? kDefaultSplitBudget : (b > 4.0 ? 4.0 : b);
}
constexpr size_t kMaxTallyBytes = 16384;  // LDS per workgroup for pre-summed tallies
constexpr size_t kMaxTimeTallyBytes = 8192;   // time histograms up to this size go to LDS
constexpr size_t kMaxLossTallyBytes = 4096;   // loss tables up to this size go to LDS
constexpr int64_t kAutoTallyCells = 64;   // default: pre-sum tallies of at most this many cells

// 4-wide BVH node, one 128-byte line: child boxes in SoA order so that a lane
// reads the node with seven 16-byte loads.  child[i] is the traversal stack
// entry of the child itself:
//   child[i] >= 0          : inner child, node index
//   child[i] == kEmptyChild: empty slot
//   otherwise              : leaf child, ~(first << 3 | (count - 1)): triangle
//                            records [first, first + count), 1 <= count <= 8
struct alignas(128) Node4 {
  float lox[4], hix[4], loy[4], hiy[4], loz[4], hiz[4];
  int32_t child[4];
  int32_t reserved[4];
};
constexpr int32_t kEmptyChild = -1 - 0x7fffffff;
constexpr int64_t kMaxLeafFirst = int64_t(1) << 28;  // leaf ranges pack first << 3
// triangle references (triangles plus split pieces): the kernels address the
// three record copies by 32-bit byte offsets with a 24-bit multiply
constexpr int64_t kMaxReferences = int64_t(1) << 24;
static_assert(sizeof(Node4) == 128, "Node4 must be one 128-byte line");

// Triangle record in leaf order, three 16-byte vectors:
//   a = (v0, bits(mesh triangle index)), b = (v1, bits(packed media/surface)),
//   c = (v2, bits(sensor id)); packed = mat_in | mat_out << 8 | (surface + 1) << 16.
// The n records are stored three times, once per dominant ray axis kz, with
// the coordinates of every vertex rotated to (kz + 1, kz + 2, kz) mod 3: the
// copy for kz starts at record ((kz + 1) mod 3) * n, so copy 0 (kz = z) is the
// mesh frame.  The ray/triangle test then reads the coordinates in the order
// it uses them instead of selecting them per test.
struct alignas(16) TriRec {
  float a[4], b[4], c[4];
};
static_assert(sizeof(TriRec) == 48, "TriRec is 48 bytes");

struct DevMaterial {
  float n, abs_len, ray_len, pad;
};

// Surface: an explicit partition as cumulative thresholds of one uniform
// draw, or (model != 0) a complex-index / thin-film reflector.
struct DevSurface {
  float c_detect, c_absorb, c_diffuse, c_specular;  // cumulative sums, rounded once
  float p_transmit, inv_r, inv_t;                    // 1/(R_diff+R_spec), 1/T
  int32_t flags_grad;                                // flags | (grad_param + 1) << 8
  int32_t model;                                     // XP_SURF_*
  float n_re, n_im, film_n, two_pi_d;                // 2 pi film thickness (nm)
};

constexpr int kMaxDispersion = 8;
// Material dispersion table: samples at ascending wavelengths of the index
// and of the attenuation coefficients 1/L_abs, 1/L_Rayleigh (0: no process).
struct DevDispersion {
  int32_t n;
  float lambda[kMaxDispersion], index[kMaxDispersion];
  float inv_abs[kMaxDispersion], inv_ray[kMaxDispersion];
};

// kForwardTally: the forward transport with its hit-map and gradient tallies
// pre-summed per workgroup in LDS (a separate instantiation, so the plain
// forward kernel carries none of its registers)
enum Mode : int32_t { kForward = 0, kBackward = 1, kForwardTally = 2 };

// Everything a propagate launch needs, passed by value (kernel arguments).
struct LaunchArgs {
  const Node4* nodes;
  const TriRec* tris;
  const int32_t* channel_of_sensor;
  int32_t n_tris;          // triangle references (records per rotated copy)
  int32_t n_lds_nodes;
  int32_t stack_lds;       // LDS window entries per lane (power of two)
  int32_t stack_total;     // worst-case stack entries of the BVH
  int32_t* stack_overflow; // [stack_total][grid * block] spill slots
  int32_t n_channels;
  int32_t n_sensors;
  // sources
  int32_t src_kind, medium;
  int64_t n_photons, n_sources;
  const float* positions;
  const int64_t* offsets;
  int64_t count_per_source;
  int32_t per_source_events;
  int32_t chunk;
  int32_t wave_batch;      // lanes not searching before a wave runs its interaction phase
  // per-event hit maps with prefix offsets and at most 64 channels: each wave
  // sums the rows of its two most recent events in LDS (event_cache 1), and
  // the first n_big_chunks chunks of kBigChunk ids go out before the rest in
  // chunks of `chunk` ids, so that a wave sees many photons of one event
  int32_t event_cache;
  int64_t n_big_chunks;
  const float* dirs;
  const float* pols;
  float cyl_r, cyl_zlo, cyl_zhi;
  int32_t time_profile;    // XP_TIME_*
  float tau_singlet, tau_triplet, singlet_fraction;
  float wl_mean, wl_sigma; // emission spectrum (sigma 0: one line)
  int32_t dispersive;      // bit m: material m has a dispersion table
  // run parameters
  uint32_t seed_lo, seed_hi;
  uint64_t pid_base;
  int32_t max_steps;
  float eps;
  int32_t grad_material;
  float surface_offset;
  // outputs
  int32_t* hit_map;
  double* grad;
  xp_photon_record* records;
  unsigned long long* stats;
  unsigned long long* work_counter;
  const float* grad_hits;  // backward: upstream gradient per hit-map cell
  double* grad_params;     // backward: 4 accumulated parameter gradients
  int32_t* time_hist;      // [events][n_time_bins] detected photons by arrival time
  int32_t n_time_bins;
  float time_inv_bin;      // 1 / bin width (ns^-1), rounded once on the host
  unsigned long long* loss;  // [n_groups + materials][8] photons by end place and flag
  const int32_t* tri_group;  // loss group of each mesh triangle
  int32_t n_groups;
  DevMaterial mats[kMaxMaterials];
  DevSurface surfs[kMaxSurfaces];
  DevDispersion disp[kMaxMaterials];
  // per-workgroup LDS tallies (kForwardTally launches)
  int32_t tally_cells;     // hit-map (and gradient) cells summed in LDS, 0: device memory
  int32_t tally_bytes;     // LDS bytes of all block tallies (a multiple of 128)
  int32_t lds_time_off;    // byte offset of the time histogram in LDS, < 0: device memory
  int32_t lds_loss_off;    // byte offset of the loss table in LDS, < 0: device memory
  int32_t n_time_cells;    // events * time bins
  int32_t n_loss_cells;    // (groups + materials) * 8
};

struct BvhResult {
  std::vector<Node4> nodes;
  std::vector<TriRec> tris;        // 3 * n_refs records: the three rotated copies
  int64_t n_refs = 0;              // triangle references (records per copy)
  int32_t depth = 0;
  int32_t max_stack = 0;
  std::vector<int32_t> level_end;  // level_end[l] = number of nodes in levels 0..l
};

// Host BVH build: binned SAH binary tree collapsed to 4-wide nodes in
// breadth-first order; triangle records in leaf order.  Returns false and an
// error message on failure.
bool build_bvh4(const float* vtx, const int32_t* tri, int64_t nt, const int32_t* mat_in,
                const int32_t* mat_out, const int32_t* surface, const int32_t* sensor,
                int max_leaf, int bins, double split_budget, BvhResult& out, std::string& err);

// Fixed device scratch of the allocation-free entry point (defined in the
// kernel translation unit): the work counter in its first 256 bytes, the
// traversal-stack overflow area after it.  scratch_init (once per device,
// with that device current) looks up the array's device address;
// scratch_base returns it (nullptr before scratch_init on that device).
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr size_t kScratchCounterBytes = 256;
hipError_t scratch_init(int device);
void* scratch_base(int device);

// Launch wrappers (defined in the kernel translation unit).
hipError_t launch_reset(unsigned long long* counter, hipStream_t s);
hipError_t launch_propagate(const LaunchArgs& a, int mode, bool grad, bool records, bool count,
                            int block, int grid, hipStream_t s);
hipError_t max_blocks_per_cu(int block, size_t lds_bytes, bool count, bool tally, int* out);
// the kForwardTally variants (compiled apart, in propagate_tally.hip)
hipError_t launch_propagate_tally(const LaunchArgs& a, bool grad, bool offsets, int block,
                                  int grid, size_t lds, hipStream_t s);
hipError_t max_blocks_per_cu_tally(int block, size_t lds_bytes, int* out);
// LDS bytes of the per-workgroup tallies (a multiple of 16)
__host__ __device__ inline size_t tally_lds_bytes(int32_t cells, bool grad) {
  return cells > 0 ? (size_t(cells) * (grad ? 40 : 4) + 15) & ~size_t(15) : 0;
}
size_t propagate_lds_bytes(int32_t n_lds_nodes, int32_t stack_lds, int block, size_t tally_bytes);
hipError_t launch_closest_hit(const Node4* nodes, const TriRec* tris, int32_t n_tris,
                              int32_t stack_depth, int64_t n, const float* orig, const float* dir,
                              const int32_t* skip, float tmin, float tmax, int32_t brute,
                              int32_t* out_tri, float* out_t, hipStream_t s);
hipError_t launch_sample(int32_t kind, uint64_t seed, uint64_t pid0, int64_t n, const float* in_dir,
                         const float* in_pol, float cyl_r, float zlo, float zhi, float* out_dir,
                         float* out_pol, hipStream_t s);
hipError_t launch_emission_time(uint64_t seed, uint64_t pid0, int64_t n, float tau_singlet,
                                float tau_triplet, float singlet_fraction, float* out_t,
                                int32_t* out_singlet, hipStream_t s);
hipError_t launch_time_quantile(const int32_t* hist, int64_t n_events, int32_t n_bins,
                                float bin_ns, float q, float* out, hipStream_t s);
hipError_t launch_valu_probe(int32_t kind, float m, float c, int32_t iters, int32_t blocks,
                             float* out, hipStream_t s);
hipError_t launch_stream_read(const void* buf, int64_t n_vec, int32_t passes, int32_t blocks,
                              float* out, hipStream_t s);
hipError_t launch_wavelength(uint64_t seed, uint64_t pid0, int64_t n, float mean, float sigma,
                             float* out, hipStream_t s);
hipError_t launch_reflectance(int32_t model, float n1, float n_re, float n_im, float film_n,
                              float two_pi_d, float lambda, int64_t n, const float* cos_i,
                              float* out_rs, float* out_rp, hipStream_t s);

}  // namespace xp

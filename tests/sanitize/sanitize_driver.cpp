// Host-side sanitizer driver (test infrastructure): built with AddressSanitizer
// and UndefinedBehaviorSanitizer on the host code only, it runs the library's
// host BVH build and argument checks and the oracle's transport over scenes
// that the test writes to disk.  Any sanitizer report aborts the process.
//
//   sanitize_driver bvh <scene> <leaf:split>...   host BVH builds (leaf size, split budget)
//   sanitize_driver oracle <scene> <n> <brute|bvh>...  oracle transport of n photons
//   sanitize_driver api                            argument and state checks that need no device
//
// Scene file (little-endian): int64 nv, nt, n_mats, n_surfs, n_sensors, n_channels;
// float vtx[3 nv]; int32 tri[3 nt], mat_in[nt], mat_out[nt], surface[nt], sensor[nt];
// float mats[3 n_mats], surf_p[5 n_surfs]; int32 surf_tags[3 n_surfs];
// float surf_optics[4 n_surfs]; int32 channel[n_sensors];
// float cyl[3] (radius, z_lo, z_hi of the uniform source volume).
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "xephot.h"

extern "C" {
struct OracleRecord {
  int32_t flag, last_tri, sensor, steps, event, medium, n_scatter, pad;
  double pos[3], dir[3], pol[3], time, path_len, sum_inv_r, sum_inv_t, wavelength;
};
void* oracle_scene_create(const float*, int64_t, const int32_t*, int64_t, const int32_t*,
                          const int32_t*, const int32_t*, const int32_t*, const float*, int32_t,
                          const float*, const int32_t*, const float*, int32_t, const int32_t*,
                          int32_t, int32_t, int32_t);
void oracle_scene_destroy(void*);
int oracle_run(void*, int32_t, int32_t, int64_t, int64_t, const float*, const int64_t*, int64_t,
               int32_t, const float*, const float*, double, double, double, int32_t, double,
               double, double, double, double, uint64_t, uint64_t, int32_t, double, int32_t,
               double, int64_t, int64_t, OracleRecord*, int64_t*, double*, int32_t);
}

namespace {

struct Scene {
  int64_t nv = 0, nt = 0, n_mats = 0, n_surfs = 0, n_sensors = 0, n_channels = 0;
  std::vector<float> vtx, mats, surf_p, surf_optics, cyl;
  std::vector<int32_t> tri, mat_in, mat_out, surface, sensor, surf_tags, channel;
};

template <class T>
void read_into(FILE* f, std::vector<T>& v, int64_t n) {
  v.resize(size_t(n));
  if (n > 0 && std::fread(v.data(), sizeof(T), size_t(n), f) != size_t(n)) {
    std::fprintf(stderr, "short scene file\n");
    std::exit(2);
  }
}

Scene load(const char* path) {
  FILE* f = std::fopen(path, "rb");
  if (!f) {
    std::fprintf(stderr, "cannot open %s\n", path);
    std::exit(2);
  }
  Scene s;
  int64_t h[6];
  if (std::fread(h, sizeof(int64_t), 6, f) != 6) std::exit(2);
  s.nv = h[0]; s.nt = h[1]; s.n_mats = h[2]; s.n_surfs = h[3]; s.n_sensors = h[4];
  s.n_channels = h[5];
  read_into(f, s.vtx, 3 * s.nv);
  read_into(f, s.tri, 3 * s.nt);
  read_into(f, s.mat_in, s.nt);
  read_into(f, s.mat_out, s.nt);
  read_into(f, s.surface, s.nt);
  read_into(f, s.sensor, s.nt);
  read_into(f, s.mats, 3 * s.n_mats);
  read_into(f, s.surf_p, 5 * s.n_surfs);
  read_into(f, s.surf_tags, 3 * s.n_surfs);
  read_into(f, s.surf_optics, 4 * s.n_surfs);
  read_into(f, s.channel, s.n_sensors);
  read_into(f, s.cyl, 3);
  std::fclose(f);
  return s;
}

int fail(const char* what) {
  std::fprintf(stderr, "FAILED: %s\n", what);
  return 1;
}

int run_bvh(const Scene& s, int n_specs, char** specs) {
  for (int k = 0; k < n_specs; ++k) {
    struct { int leaf; float split; } o{1, 0.0f};
    if (std::sscanf(specs[k], "%d:%f", &o.leaf, &o.split) != 2) return fail("bad leaf:split");
    xp_bvh_options bo{o.leaf, 32, o.split};
    xp_bvh_info info{};
    if (xp_bvh_build_host(s.vtx.data(), s.nv, s.tri.data(), s.nt, &bo, &info, nullptr, 0, nullptr,
                          0) != XP_OK)
      return fail(xp_last_error(nullptr));
    std::vector<unsigned char> nodes(size_t(info.n_nodes) * 128), recs(size_t(3 * info.n_references) * 48);
    if (xp_bvh_build_host(s.vtx.data(), s.nv, s.tri.data(), s.nt, &bo, &info, nodes.data(),
                          info.n_nodes, recs.data(), 3 * info.n_references) != XP_OK)
      return fail(xp_last_error(nullptr));
    if (info.n_references < s.nt) return fail("fewer references than triangles");
    // buffers one element short must be refused, not overrun
    if (info.n_nodes > 1 &&
        xp_bvh_build_host(s.vtx.data(), s.nv, s.tri.data(), s.nt, &bo, &info, nodes.data(),
                          info.n_nodes - 1, recs.data(), 3 * info.n_references) == XP_OK)
      return fail("short node buffer accepted");
    std::printf("bvh leaf %d split %g: %lld nodes, %lld references, depth %d, stack %d\n", o.leaf,
                double(o.split), (long long)info.n_nodes, (long long)info.n_references, info.depth,
                info.max_stack);
  }
  return 0;
}

int run_oracle(const Scene& s, int64_t n, int n_modes, char** modes) {
  for (int k = 0; k < n_modes; ++k) {
    const int bvh = std::strcmp(modes[k], "bvh") == 0 ? 1 : 0;
    void* sc = oracle_scene_create(s.vtx.data(), s.nv, s.tri.data(), s.nt, s.mat_in.data(),
                                   s.mat_out.data(), s.surface.data(), s.sensor.data(),
                                   s.mats.data(), int32_t(s.n_mats), s.surf_p.data(),
                                   s.surf_tags.data(), s.surf_optics.data(), int32_t(s.n_surfs),
                                   s.channel.data(), int32_t(s.n_sensors),
                                   int32_t(s.n_channels), bvh);
    std::vector<OracleRecord> rec(static_cast<size_t>(n));
    std::vector<int64_t> hits(size_t(std::max<int64_t>(s.n_channels, 1)), 0);
    std::vector<double> grad(hits.size() * 4, 0.0);
    // uniform-cylinder sources with the scintillation profile and the
    // Gaussian spectrum, gradient tallies for material 0
    const int rc = oracle_run(sc, 1, 0, n, 0, nullptr, nullptr, 0, 0, nullptr, nullptr, s.cyl[0],
                              s.cyl[1], s.cyl[2], 1, 3.5, 24.0, 0.66, 174.8, 10.2, 7, 0, 10000,
                              0.0, 0, 2e-6, 0, n, rec.data(), hits.data(), grad.data(), 1);
    if (rc != 0) return fail("oracle_run");
    int64_t total = 0;
    for (int64_t h : hits) total += h;
    int64_t ended = 0;
    for (const auto& r : rec) ended += (r.flag & 0xff) >= 1 && (r.flag & 0xff) <= 7;
    if (ended != n) return fail("a photon without a terminal flag");
    std::printf("oracle %s: %lld photons, %lld detected\n", bvh ? "bvh" : "brute",
                (long long)n, (long long)total);
    oracle_scene_destroy(sc);
  }
  return 0;
}

int run_api() {
  xp_context* ctx = nullptr;
  // without a device the context cannot be made; the error must be reported
  const int rc = xp_context_create(0, &ctx);
  if (rc == XP_OK) {
    // a device is present: exercise the state checks on an empty context
    if (xp_build_bvh(ctx, nullptr) == XP_OK) return fail("BVH built without a mesh");
    xp_sources src{};
    xp_run_params rp{};
    if (xp_propagate(ctx, &src, &rp, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) ==
        XP_OK)
      return fail("propagate without a BVH");
    xp_context_destroy(ctx);
  } else if (ctx != nullptr || std::strlen(xp_last_error(nullptr)) == 0) {
    return fail("context failure not reported");
  }
  if (xp_propagate(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                   nullptr) == XP_OK)
    return fail("null context accepted");
  if (xp_time_quantile(nullptr, 4, 8, 1.0f, 0.9f, nullptr, nullptr) == XP_OK)
    return fail("time quantile without buffers accepted");
  if (xp_sample(7, 0, 0, 10, nullptr, nullptr, 0, 0, 0, nullptr, nullptr, nullptr) == XP_OK)
    return fail("unknown sampler accepted");
  // malformed meshes: out-of-range index, non-finite coordinate, degenerate triangle
  const float v[12] = {0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, NAN};
  const int32_t bad_index[3] = {0, 1, 5}, nan_vertex[3] = {0, 1, 3}, degenerate[3] = {0, 1, 1};
  xp_bvh_info info{};
  for (const int32_t* t : {bad_index, nan_vertex, degenerate})
    if (xp_bvh_build_host(v, 4, t, 1, nullptr, &info, nullptr, 0, nullptr, 0) == XP_OK)
      return fail("malformed mesh accepted");
  std::printf("api checks passed (%s)\n", xp_version());
  return 0;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc >= 4 && !std::strcmp(argv[1], "bvh")) return run_bvh(load(argv[2]), argc - 3, argv + 3);
  if (argc >= 5 && !std::strcmp(argv[1], "oracle"))
    return run_oracle(load(argv[2]), std::atoll(argv[3]), argc - 4, argv + 4);
  if (argc >= 2 && !std::strcmp(argv[1], "api")) return run_api();
  std::fprintf(stderr, "usage: sanitize_driver bvh|oracle|api ...\n");
  return 2;
}

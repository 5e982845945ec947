/*
 * xephot.h -- C ABI of the MI355X (gfx950) optical-photon transport library.
 *
 * The library propagates batches of monochromatic scintillation photons
 * (175 nm) through a triangle-mesh detector and tallies the photons detected
 * by each photosensor, as the paper's optical simulation of the DARWIN TPC
 * does (sections "Simulation of the DARWIN detector" and "Optical
 * properties", table tab:optical).  Processes: bulk absorption (absorption
 * length), Rayleigh scattering (dipole law, appendix item 3), explicit
 * angle-independent surfaces split into detect / absorb / diffuse / specular /
 * transmit, Fresnel reflection and refraction with total internal reflection
 * at boundaries between dielectrics (quartz, LXe, GXe), and detection at
 * sensors (the LCE definition of section "Comparison of Chroma and Geant4").
 *
 * Conventions for every entry point:
 *  - Units: metres and nanoseconds.
 *  - Return value: XP_OK (0) or a negative xp_status.  No C++ exception
 *    crosses this boundary.  xp_last_error() gives a message.
 *  - Arguments documented "host" are read during the call and may be freed
 *    after it returns.  Arguments documented "device" are device memory on the
 *    context's GPU, owned by the caller, and must stay alive until the work
 *    queued on the given stream has completed.
 *  - Per-photon physics failures are not errors: every photon ends with one
 *    terminal flag (XP_FLAG_*), visible in the optional per-photon records.
 *  - A context may be used from one host thread at a time.
 */
#ifndef XEPHOT_H_
#define XEPHOT_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct xp_context xp_context;
typedef void* xp_stream; /* a hipStream_t (0 = the null stream) */

typedef enum xp_status {
  XP_OK = 0,
  XP_ERR_INVALID_ARG = -1, /* a null pointer, a size or an id out of range */
  XP_ERR_STATE = -2,       /* call out of order (e.g. propagate before build_bvh) */
  XP_ERR_MESH = -3,        /* mesh failed validation */
  XP_ERR_HIP = -4,         /* a HIP runtime call failed */
  XP_ERR_OOM = -5,         /* device or host allocation failed */
  XP_ERR_UNSUPPORTED = -6  /* valid request the library cannot serve (e.g. BVH too deep) */
} xp_status;

/* Terminal flags of a photon (low byte) plus the GEOMETRY_ERROR bit. */
enum {
  XP_FLAG_DETECT = 1,         /* collected by a sensor (counted in the hit map) */
  XP_FLAG_SENSOR_ABSORB = 2,  /* reached a sensor's active face, not detected (QE miss) */
  XP_FLAG_SURFACE_ABSORB = 3, /* absorbed by a surface (or the back of a front-only sensor) */
  XP_FLAG_BULK_ABSORB = 4,    /* absorbed in the medium */
  XP_FLAG_ESCAPED = 5,        /* no triangle ahead and no bulk process (mesh leak) */
  XP_FLAG_MAX_STEPS = 6,      /* still alive after max_steps steps */
  XP_FLAG_NAN_ABORT = 7,      /* a non-finite position or direction */
  XP_FLAG_GEOMETRY_ERROR = 0x100 /* arrived from a medium other than the tracked one */
};

/* ------------------------------------------------------------------------- */
/* context                                                                    */
/* ------------------------------------------------------------------------- */

/* Create a context on HIP device `hip_device`.  *out receives the handle.
 * The library owns every device copy of geometry and tables it makes; they are
 * freed by xp_context_destroy.  Errors: XP_ERR_INVALID_ARG, XP_ERR_HIP. */
int xp_context_create(int hip_device, xp_context** out);
void xp_context_destroy(xp_context* ctx);

/* Message of the last failed call on ctx, valid until the next call on ctx;
 * xp_last_error(NULL) gives the calling thread's last message (used when
 * xp_context_create fails).  Never NULL. */
const char* xp_last_error(const xp_context* ctx);

/* ------------------------------------------------------------------------- */
/* geometry and optical tables (the paper's per-component optical properties,
 * table tab:optical)                                                         */
/* ------------------------------------------------------------------------- */

/* Load an indexed triangle mesh (host arrays, copied).
 *   vtx        float[nv*3]  vertex coordinates (m)
 *   tri        int32[nt*3]  vertex indices; the geometric normal
 *                           (v1-v0) x (v2-v0) points to the triangle's OUTER side
 *   mat_inner  int32[nt]    material on the inner side, mat_outer on the outer
 *   surface    int32[nt]    surface id, or -1: no explicit surface (a Fresnel
 *                           boundary when the refractive indices differ, else
 *                           the photon passes through)
 *   sensor     int32[nt]    sensor id, or -1
 * Validation: nv, nt > 0, nt < 2^31; indices in [0, nv); finite coordinates;
 * triangle area >= 1e-12 m^2; material ids in [0, 255]; surface ids in
 * [-1, 65534]; sensor ids >= -1.  Errors: XP_ERR_INVALID_ARG, XP_ERR_MESH.
 * Replaces any previous mesh and invalidates the BVH. */
int xp_load_mesh(xp_context* ctx, const float* vtx, int64_t nv, const int32_t* tri, int64_t nt,
                 const int32_t* mat_inner, const int32_t* mat_outer, const int32_t* surface,
                 const int32_t* sensor);

/* Bulk optical properties of a medium.  Lengths may be INFINITY (no process). */
typedef struct xp_material {
  float n;                 /* real refractive index */
  float abs_length;        /* absorption length L_abs (m), > 0 */
  float rayleigh_length;   /* Rayleigh scattering length L_Rayleigh (m), > 0 */
} xp_material;

/* Set the material table (host array of n <= 8 entries, copied).  Clears
 * every dispersion table.
 * Errors: XP_ERR_INVALID_ARG (n out of range, a non-positive or NaN value). */
int xp_set_materials(xp_context* ctx, const xp_material* m, int32_t n);

/* Wavelength dependence of material `material` (section "Optical
 * properties": the paper tabulates its values at the mean of the emission
 * spectrum): n_points <= 8 samples at ascending wavelengths lambda_nm (host
 * arrays, copied) of the index and of the absorption and Rayleigh lengths (m,
 * INFINITY allowed).  At a photon's wavelength the index and the attenuation
 * coefficients 1/L are interpolated linearly between the two neighbouring
 * samples and held constant outside them; the material's table entry is then
 * not used.  n_points = 0 removes the table.  Gradient tallies and the
 * backward pass reject a gradient material that has a table.
 * Errors: XP_ERR_STATE (material not set), XP_ERR_INVALID_ARG. */
int xp_set_material_dispersion(xp_context* ctx, int32_t material, int32_t n_points,
                               const float* lambda_nm, const float* index,
                               const float* abs_length, const float* rayleigh_length);

#define XP_SURF_DETECT_FRONT_ONLY 1 /* detect only photons arriving from the outer side;
                                       from the inner side the surface absorbs */

/* Surface models.
 * EXPLICIT: the probabilities partition [0, 1) in the order
 *   detect | absorb | diffuse (Lambertian) | specular | transmit, independent of
 *   the angle of incidence; any rounding remainder absorbs.  `grad_param` tags
 *   the surface for the gradient tallies: 2 = reflectivity parameter (scales
 *   the diffuse and specular parts together), 3 = transparency parameter, -1
 *   none.
 * COMPLEX_INDEX: behind the surface lies a medium of complex index
 *   n_re + i n_im (n_im >= 0: absorbing), e.g. the silicon of the 4-pi design's
 *   optical table (0.81 + 1.86 i).  THIN_FILM: a dielectric film of index
 *   film_n and thickness film_thickness_nm on such a medium (an Al/MgF2
 *   coating).  For both, a photon arriving from a medium of index n1 is
 *   reflected specularly with probability a_s^2 |r_s|^2 + a_p^2 |r_p|^2 (a_s,
 *   a_p: components of its linear polarization along s and p; amplitude
 *   coefficients in the Born and Wolf convention with q = sqrt(n^2 - n1^2
 *   sin^2), principal branch, and the film phase 2 pi d q_film / lambda at the
 *   photon's wavelength); the reflected photon stays linearly polarized, its s
 *   and p components scaled by |r| with the sign of Re r.  A photon not
 *   reflected is detected if the triangle is a sensor, else absorbed.  The
 *   probability fields are ignored; grad_param must be -1. */
enum { XP_SURF_EXPLICIT = 0, XP_SURF_COMPLEX_INDEX = 1, XP_SURF_THIN_FILM = 2 };

typedef struct xp_surface {
  float p_detect, p_absorb, r_diffuse, r_specular, p_transmit;
  int32_t grad_param;
  int32_t flags;           /* XP_SURF_DETECT_FRONT_ONLY */
  int32_t model;           /* XP_SURF_EXPLICIT / COMPLEX_INDEX / THIN_FILM */
  float n_re, n_im;        /* complex index behind the surface */
  float film_n;            /* THIN_FILM: film index (> 0) */
  float film_thickness_nm; /* THIN_FILM: film thickness (>= 0) */
} xp_surface;

/* Set the surface table (host array of n <= 16 entries, copied).  An
 * EXPLICIT entry's probabilities must be in [0, 1] and sum to 1 +- 1e-6; a
 * COMPLEX_INDEX or THIN_FILM entry needs finite n_re > 0, n_im >= 0 (and
 * film_n > 0, film_thickness_nm >= 0).
 * Errors: XP_ERR_INVALID_ARG. */
int xp_set_surfaces(xp_context* ctx, const xp_surface* s, int32_t n);

/* Map sensor ids to hit-map columns (host array, copied): detections on
 * sensor k count into column channel_of_sensor[k] of n_channels.  Without a
 * call the map is the identity with n_channels = 1 + the largest sensor id.
 * Errors: XP_ERR_INVALID_ARG (a column outside [0, n_channels)). */
int xp_set_channel_map(xp_context* ctx, const int32_t* channel_of_sensor, int32_t n_sensors,
                       int32_t n_channels);

/* ------------------------------------------------------------------------- */
/* acceleration structure (the paper names none; this library's own)          */
/* ------------------------------------------------------------------------- */

typedef struct xp_bvh_options {
  int32_t max_leaf_size;   /* triangles per leaf, 1..8 (default 1: a search micro-step
                              tests one triangle and visits one node, and single-triangle
                              leaves keep the triangle tests fewest) */
  int32_t sah_bins;        /* SAH bins per axis, 4..64 (default 32) */
  float split_budget;      /* triangles whose box is more than twice the least box a planar
                              piece of their area and orientation needs (long slivers,
                              fans) are clipped into pieces with tighter boxes, the most
                              wasted box area first, adding at most this fraction of the
                              triangle count as extra references, 0..4 (0 = default: the
                              larger of 0.02 and 2048 / triangles, at most 4; negative =
                              no splitting).  Every piece refers to the whole triangle:
                              results are identical either way */
} xp_bvh_options;

typedef struct xp_bvh_stats {
  int64_t n_nodes;         /* 4-wide nodes of 128 bytes */
  int64_t n_triangles;     /* triangles of the mesh; stored as 48-byte records, one per
                              reference, in three copies (one per dominant ray axis) */
  int32_t depth;           /* levels below the root */
  int32_t max_stack;       /* worst-case traversal stack entries */
  int64_t node_bytes, triangle_bytes;
  double build_seconds;
  int64_t n_references;    /* triangle references in the leaves (n_triangles plus the
                              extra pieces of split triangles); the records are stored per
                              reference: triangle_bytes = 3 * 48 * n_references */
} xp_bvh_info;

/* Build the BVH on the host (binned SAH, collapsed to 4-wide nodes) and upload
 * it.  opts may be NULL (defaults).  Must follow xp_load_mesh
 * (else XP_ERR_STATE).  Meshes of 2^24 or more triangles are rejected
 * (XP_ERR_UNSUPPORTED: the kernels address the triangle records by 32-bit
 * byte offsets), and reference splitting stops below 2^24 references.
 * Synchronizes the
 * device.  Errors: XP_ERR_STATE, XP_ERR_INVALID_ARG, XP_ERR_MESH, XP_ERR_OOM,
 * XP_ERR_HIP, XP_ERR_UNSUPPORTED. */
int xp_build_bvh(xp_context* ctx, const xp_bvh_options* opts);
int xp_bvh_stats(const xp_context* ctx, xp_bvh_info* out);

/* The same host BVH build without a device or a context, for inspecting and
 * testing the structure the kernels traverse.  vtx / tri / nv / nt as in
 * xp_load_mesh (geometric checks only; media, surfaces and sensors are taken
 * as 0 / -1 / -1); opts as in xp_build_bvh.  Fills *info (build_seconds:
 * this call) and, when not NULL, copies
 *   nodes    info->n_nodes 128-byte nodes, breadth-first, root first:
 *            float lo_x[4], hi_x[4], lo_y[4], hi_y[4], lo_z[4], hi_z[4] (child
 *            boxes, padded outward by 2^-20 relative + 1e-7 m; an empty slot
 *            holds lo = +INFINITY, hi = -INFINITY), int32 child[4]
 *            (>= 0: inner node index; INT32_MIN: empty slot; else the
 *            complement of a leaf's first << 3 | (count - 1), a range of
 *            records), int32 reserved[4] (0);
 *   records  3 * info->n_references 48-byte records in leaf order, in three
 *            copies (copy c starts at record c * n_references and holds the
 *            coordinates rotated to (k + 1, k + 2, k) mod 3 for the dominant
 *            ray axis k = (c + 2) mod 3, so copy 0 is the mesh frame): float
 *            v0[3], int32 triangle index, float v1[3], int32 packed media and
 *            surface, float v2[3], int32 sensor id.
 * nodes_capacity counts nodes, records_capacity records; a buffer too small
 * gives XP_ERR_INVALID_ARG.  Call once with NULL buffers for the sizes.
 * Errors: XP_ERR_INVALID_ARG, XP_ERR_MESH, XP_ERR_OOM, XP_ERR_UNSUPPORTED
 * (xp_last_error(NULL)). */
int xp_bvh_build_host(const float* vtx, int64_t nv, const int32_t* tri, int64_t nt,
                      const xp_bvh_options* opts, xp_bvh_info* info, void* nodes,
                      int64_t nodes_capacity, void* records, int64_t records_capacity);

/* ------------------------------------------------------------------------- */
/* photon sources                                                             */
/* ------------------------------------------------------------------------- */

enum {
  XP_SRC_POINTS = 0,           /* isotropic point sources (the paper's point-source and
                                  Z-scan runs); photon i belongs to source s with
                                  offsets[s] <= i < offsets[s+1] */
  XP_SRC_UNIFORM_CYLINDER = 1, /* each photon at its own uniform point of the cylinder
                                  r <= cyl_radius, cyl_zlo <= z <= cyl_zhi (the average-LCE
                                  run: photons uniform in the active volume) */
  XP_SRC_EXPLICIT = 2          /* given position, direction and polarization per photon */
};

typedef struct xp_sources {
  int32_t kind;               /* XP_SRC_* */
  int32_t medium;             /* material id the photons start in */
  int64_t n_photons;          /* photons in this launch, >= 0 */
  int64_t n_sources;          /* POINTS: number of points */
  const float* positions;     /* device: POINTS float[n_sources*3]; EXPLICIT float[n_photons*3] */
  const int64_t* offsets;     /* device: POINTS int64[n_sources+1] prefix sums (offsets[0] = 0,
                                 offsets[n_sources] = n_photons), or NULL: count_per_source each */
  int64_t count_per_source;   /* POINTS without offsets */
  int32_t per_source_events;  /* POINTS: 1 = one hit-map row per source, 0 = a single row */
  int32_t reserved;
  const float* directions;    /* device: EXPLICIT float[n_photons*3] (unit) */
  const float* polarizations; /* device: EXPLICIT float[n_photons*3] (made transverse) */
  float cyl_radius, cyl_zlo, cyl_zhi; /* UNIFORM_CYLINDER */
  int32_t time_profile;       /* XP_TIME_ZERO or XP_TIME_SCINTILLATION */
  float tau_singlet_ns;       /* SCINTILLATION: decay constants (> 0) and the fraction */
  float tau_triplet_ns;       /*   of photons from the singlet state (in [0, 1]); the */
  float singlet_fraction;     /*   paper's optical table gives 3.5 ns, 24 ns, 0.66 (NR) */
  float wavelength_nm;        /* mean of the Gaussian emission spectrum (174.8 in the
                                 paper); >= 0, and > 0 when a THIN_FILM surface exists */
  float wavelength_fwhm_nm;   /* its FWHM (10.2 in the paper); 0: every photon at the
                                 mean.  Photon id pid draws (u0, u1) from Philox block
                                 (step 0, sub 3): lambda = mean + sigma sqrt(-2 ln u0)
                                 cos(2 pi u1), sigma = FWHM / (2 sqrt(2 ln 2)) */
} xp_sources;

/* Emission time of the photons (section "Optical properties": scintillation
 * as a two-component exponential decay).  ZERO: every photon starts at t = 0.
 * SCINTILLATION: photon id pid draws (u0, u1) from Philox block (step 0, sub 2);
 * it comes from the singlet state if u0 < singlet_fraction, and starts at
 * t = -tau ln(u1) with that state's decay constant. */
enum { XP_TIME_ZERO = 0, XP_TIME_SCINTILLATION = 1 };

/* ------------------------------------------------------------------------- */
/* propagation                                                                */
/* ------------------------------------------------------------------------- */

typedef struct xp_run_params {
  uint64_t seed;           /* Philox-4x32-10 key */
  uint64_t pid_base;       /* photon i of this launch has id pid_base + i; its random
                              numbers depend only on (seed, id) */
  int32_t max_steps;       /* steps before XP_FLAG_MAX_STEPS (default 10000 if <= 0) */
  float eps;               /* hits on triangles other than the last one are taken for
                              distances > eps (m); 0 is the default */
  int32_t grad_material;   /* material whose L_abs / L_Rayleigh are gradient params 0 / 1
                              (-1: none) */
  float surface_offset;    /* m: after a surface interaction the photon restarts this far
                              from the surface along its normal, on the side it leaves
                              toward (recommended 2e-6: above the FP32 rounding of
                              positions up to ~3 m, below any feature of the meshes) */
} xp_run_params;

typedef struct xp_launch_cfg {
  int32_t block_size;      /* threads per workgroup: 64, 128 or 256 (0 = default) */
  int32_t blocks_per_cu;   /* resident workgroups per CU (0 = as many as fit) */
  int32_t chunk;           /* photon ids claimed per wave refill (0 = default 64) */
  int32_t lds_levels;      /* BVH levels staged in LDS, 0..4; -1 = automatic: four,
                              or three where the fourth would lower the occupancy or
                              leave the launch's LDS tallies (block_tally) no room */
  int32_t stack_lds;       /* traversal-stack entries per lane kept in LDS, a power of
                              two in 4..64 (0 = default 16); when a node visit would
                              leave fewer than four of them free, the lane's LDS entries
                              move to a global overflow area allocated by xp_build_bvh */
  int32_t wave_batch;      /* photons per wave interaction phase: a wave interrupts its
                              closest-hit searches to run the interactions, tallies and
                              refills once at least this many of its 64 lanes are not
                              searching, 1..64 (0 = default 32) */
  int32_t block_tally;     /* tallies of a launch without records or counters, summed
                              per workgroup in LDS and added to device memory once per
                              workgroup (when they fit without lowering the occupancy)
                              instead of one device-memory atomic per photon: 1 = the hit
                              map and gradients at any size that fits; 0 = default (hit
                              map and gradients for at most 64 cells); with 0 or 1 the
                              loss table (up to 4 KB) and the arrival-time histogram (up
                              to 8 KB) too; -1 = none.  Integer tallies are identical
                              either way; gradients differ only in summation order */
} xp_launch_cfg;

/* One per photon (indexed by the launch-local photon index), written when
 * requested.  96 bytes.  The score inputs (n_scatter, path_len, sum_inv_r,
 * sum_inv_t) are tracked only by launches that also tally gradients
 * (d_grad != NULL); otherwise they are 0. */
typedef struct xp_photon_record {
  int32_t flag, last_tri, sensor, steps;
  int32_t event, medium, n_scatter, reserved;
  float pos[3];  float time;       /* final position (m), time of flight (ns) */
  float dir[3];  float path_len;   /* final direction; path length in grad_material */
  float pol[3];  float sum_inv_r;  /* final polarization; sum of 1/R over tagged reflections */
  float sum_inv_t; float wavelength; /* sum of 1/T over tagged transmissions; nm */
  float pad[2];
} xp_photon_record;

/* Launch the transport of src->n_photons photons on `stream` (asynchronous).
 *   d_hit_map  device int32 [n_events * n_channels], ACCUMULATED (the caller
 *              zeroes it); n_events = n_sources if per_source_events else 1.
 *              May be NULL.
 *   d_grad     device double [n_events * n_channels * 4] or NULL: accumulates,
 *              per detected photon, its score-function weights for
 *              (L_abs, L_Rayleigh of grad_material, reflectivity, transparency),
 *              i.e. the Jacobian of the expected hits.
 *   d_records  device xp_photon_record [n_photons] or NULL.
 *   d_stats    device uint64 [24] or NULL: ACCUMULATES counters
 *              [0..7] photons per terminal flag (index = flag low byte),
 *              [8] GEOMETRY_ERROR photons, [9] steps, [10] BVH nodes visited,
 *              [11] triangles tested, [12] search lane-slots offered and
 *              [13] used (SIMD utilization of the search), [14] reserved (0),
 *              [15] wave interaction phases,
 *              [16] / [17] wave clock cycles spent in interaction phases / in
 *              search micro-steps (counting mode costs time).
 *   lc         NULL = the context's tuned or default configuration.
 * Errors: XP_ERR_STATE (no BVH / tables), XP_ERR_INVALID_ARG, XP_ERR_HIP.
 * Concurrency: eager calls on one context use a ring of 64 work counters; at
 * most 64 eager launches of one context may be in flight at a time.  A launch
 * captured into a HIP graph (the stream is capturing) gets a work counter no
 * other launch uses, so its replays may run beside eager launches of the same
 * context on other streams; replays of one graph must not overlap each
 * other.  At most 256 launches per context may be captured
 * (XP_ERR_UNSUPPORTED beyond). */
int xp_propagate(xp_context* ctx, const xp_sources* src, const xp_run_params* rp,
                 int32_t* d_hit_map, double* d_grad, xp_photon_record* d_records,
                 uint64_t* d_stats, const xp_launch_cfg* lc, xp_stream stream);

/* Extra tallies of xp_propagate_ex (section "Light collection efficiency":
 * arrival times and t90; section "Sources of photon losses": where photons
 * end).  Every pointer may be NULL; buffers are caller-owned device memory
 * and are ACCUMULATED (the caller zeroes them).
 *   d_time_hist  int32 [n_events * n_time_bins]: detected photons by arrival
 *                time (emission time plus time of flight); bin b holds times
 *                in [b, b + 1) * time_bin_ns, the last bin also every later one.
 *                Bin index = floor(time * inv) in FP32 with
 *                inv = (float)(1.0 / time_bin_ns).
 *   d_loss       uint64 [(n_groups + n_materials) * 8], needs
 *                xp_set_loss_groups: photons by where they ended (row) and
 *                terminal flag (column = flag low byte).  Photons ending on a
 *                surface (DETECT, SENSOR_ABSORB, SURFACE_ABSORB) count in the
 *                row of their last triangle's group; all others (BULK_ABSORB,
 *                ESCAPED, MAX_STEPS, NAN_ABORT) in row n_groups + the material
 *                they were in. */
typedef struct xp_extra_tallies {
  int32_t* d_time_hist;
  int32_t n_time_bins;     /* >= 1 when d_time_hist is set */
  float time_bin_ns;       /* > 0 when d_time_hist is set */
  uint64_t* d_loss;
} xp_extra_tallies;

/* xp_propagate with the extra tallies (extra may be NULL: same as
 * xp_propagate).  Errors as xp_propagate; XP_ERR_STATE if d_loss is set and no
 * loss groups are. */
int xp_propagate_ex(xp_context* ctx, const xp_sources* src, const xp_run_params* rp,
                    int32_t* d_hit_map, double* d_grad, xp_photon_record* d_records,
                    uint64_t* d_stats, const xp_extra_tallies* extra, const xp_launch_cfg* lc,
                    xp_stream stream);

/* xp_propagate for callers that cannot allocate device memory during the call
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same launch and the same results, but the work counter and
 * the traversal-stack overflow area live in a fixed 64 MiB device array that
 * the library holds on every device it runs on until the process ends (its
 * address is looked up once per device by xp_context_create).  The call
 * allocates nothing; inputs and outputs are as in xp_propagate.  The overflow
 * area needs 4 * max_stack bytes per lane (xp_bvh_info.max_stack) for every
 * lane of the launch: with lc NULL or lc->blocks_per_cu 0 the call runs fewer
 * workgroups per CU when the default would not fit (results do not depend on
 * it); a launch that does not fit with the caller's blocks_per_cu, or with one
 * workgroup per CU, fails with XP_ERR_UNSUPPORTED.  Every call on one device
 * shares that device's array: calls that overlap in time on one device (other
 * streams, other contexts, other threads) race and give wrong results; the
 * caller serializes them.  Errors: as xp_propagate, plus XP_ERR_UNSUPPORTED
 * (scratch too small for the launch). */
int xp_propagate_static(xp_context* ctx, const xp_sources* src, const xp_run_params* rp,
                        int32_t* d_hit_map, double* d_grad, xp_photon_record* d_records,
                        uint64_t* d_stats, const xp_launch_cfg* lc, xp_stream stream);

/* Loss group of every mesh triangle (host int32 [n_triangles], mesh order,
 * copied; values in [0, n_groups)), e.g. the detector component it belongs to.
 * Must follow xp_load_mesh.  Errors: XP_ERR_STATE, XP_ERR_INVALID_ARG,
 * XP_ERR_OOM, XP_ERR_HIP. */
int xp_set_loss_groups(xp_context* ctx, const int32_t* group_of_triangle, int32_t n_groups);

/* Per-event arrival-time quantile from a time histogram (device arrays, no
 * context): d_out[e] = the time by which a fraction q of event e's detected
 * photons had arrived (q = 0.9: the paper's t90), interpolating linearly
 * inside the bin where the cumulative count reaches q * total; NaN for an
 * event with no photons, +INFINITY when the quantile falls in the last
 * (open-ended) bin.  0 < q <= 1.  Errors: XP_ERR_INVALID_ARG, XP_ERR_HIP
 * (xp_last_error(NULL)). */
int xp_time_quantile(const int32_t* d_time_hist, int64_t n_events, int32_t n_time_bins,
                     float time_bin_ns, float q, float* d_out, xp_stream stream);

/* Backward pass of the expected hit map with respect to the four parameters,
 * by replaying the same photon histories (same seed and photon ids, so no
 * path storage):  d_grad_params[p] += sum over detected photons of
 * d_grad_hits[event * n_channels + channel] * score_p.
 *   d_grad_hits    device float [n_events * n_channels]
 *   d_grad_params  device double [4], ACCUMULATED
 * Errors as xp_propagate. */
int xp_backward(xp_context* ctx, const xp_sources* src, const xp_run_params* rp,
                const float* d_grad_hits, double* d_grad_params, const xp_launch_cfg* lc,
                xp_stream stream);

/* Pick the fastest launch configuration on a sample of `src` (at most
 * sample_photons photons) by timing hit-map launches (best of three each):
 * block sizes 64 / 256, no / automatic BVH levels in LDS, 8 / 16 LDS stack
 * entries and wave_batch 16 / 32 / 48 with the default block_tally; then,
 * around the fastest so far, 2 / 3 / 4 workgroups per CU (against the
 * occupancy limit), then refill chunks of 16 / 32 / 128 / 256 photon ids
 * (against 64); then the fastest with block_tally 1 (block_tally is never set
 * to -1: the default keeps the LDS tallies that gradient launches need).  The
 * default configuration is kept unless a candidate is more than 2 % faster
 * on the sample.  Stores
 * the result in the context (used when lc is NULL) and in *out (may be
 * NULL).  Integer results never depend on the
 * choice.  Synchronizes the stream.  Errors as xp_propagate. */
int xp_autotune(xp_context* ctx, const xp_sources* src, const xp_run_params* rp,
                int64_t sample_photons, xp_launch_cfg* out, xp_stream stream);

/* ------------------------------------------------------------------------- */
/* test hooks                                                                 */
/* ------------------------------------------------------------------------- */

/* Closest hit for n rays (device arrays): orig/dir float[n*3], skip int32[n]
 * (triangle to ignore, -1 none; may be NULL); out_tri int32[n] (mesh triangle
 * index or -1), out_t float[n].  Hits are taken for t in (tmin, tmax], ties go
 * to the lower triangle index.  brute != 0 tests every triangle instead of
 * traversing the BVH. */
int xp_closest_hit(xp_context* ctx, int64_t n, const float* orig, const float* dir,
                   const int32_t* skip, float tmin, float tmax, int32_t brute, int32_t* out_tri,
                   float* out_t, xp_stream stream);

/* Device samplers (device arrays of n rows): kind 0 emission direction and
 * polarization, 1 Lambertian about in_dir, 2 Rayleigh from (in_dir, in_pol),
 * 3 uniform-cylinder positions (in out_dir).  Photon ids pid0 .. pid0+n-1 with
 * the same random-number schedule as xp_propagate. */
int xp_sample(int32_t kind, uint64_t seed, uint64_t pid0, int64_t n, const float* in_dir,
              const float* in_pol, float cyl_radius, float cyl_zlo, float cyl_zhi, float* out_dir,
              float* out_pol, xp_stream stream);

/* Emission times of photon ids pid0 .. pid0+n-1 (device float out_t[n]) and
 * their state (out_singlet int32[n]: 1 singlet, 0 triplet; may be NULL), as
 * xp_propagate draws them for XP_TIME_SCINTILLATION. */
int xp_sample_emission_time(uint64_t seed, uint64_t pid0, int64_t n, float tau_singlet_ns,
                            float tau_triplet_ns, float singlet_fraction, float* out_t,
                            int32_t* out_singlet, xp_stream stream);

/* Emission wavelengths (nm) of photon ids pid0 .. pid0+n-1 (device float
 * out[n]), as xp_propagate draws them. */
int xp_sample_wavelength(uint64_t seed, uint64_t pid0, int64_t n, float mean_nm, float fwhm_nm,
                         float* out, xp_stream stream);

/* Power reflectances |r_s|^2 and |r_p|^2 (device float out_rs[n], out_rp[n])
 * of a COMPLEX_INDEX or THIN_FILM surface at n incidence cosines (device
 * float cos_i[n]) for light from a medium of index n1 at wavelength lambda_nm,
 * as the transport evaluates them. */
int xp_surface_reflectance(int32_t model, float n1, float n_re, float n_im, float film_n,
                           float film_thickness_nm, float lambda_nm, int64_t n,
                           const float* cos_i, float* out_rs, float* out_rp, xp_stream stream);

/* Bandwidth probe for the roofline (not part of the transport): `blocks`
 * workgroups of 256 threads read the device buffer buf (n_vec 16-byte
 * vectors) `passes` times with a grid stride and write one sum per thread to
 * out (device float[blocks * 256]).  Buffers that fit the L2 caches or the
 * Infinity Cache are then read from there on every pass after the first. */
int xp_stream_read(const void* buf, int64_t n_vec, int32_t passes, int32_t blocks, float* out,
                   xp_stream stream);

/* VALU issue probe for the roofline (not part of the transport): `blocks`
 * workgroups of 256 threads each run `iters` iterations of 64 steps of one
 * kind on eight independent chains (kind 0: one FP32 multiply-add per step,
 * 1: one FP32 reciprocal, 2: a 32-bit integer xor and an add, 3: an FP32
 * multiply-add and an independent integer xor and add, 4: an FP32
 * multiply-add and an independent FP32 reciprocal, 5: a 32 x 32 -> 64-bit
 * integer multiply-add and a move) and write one value per thread to out (device
 * float[blocks * 256]).  Kernels of known instruction count for calibrating
 * the shader-sequencer counters and measuring the issue rate the chip
 * sustains for each instruction mix.  Errors: XP_ERR_INVALID_ARG,
 * XP_ERR_HIP. */
int xp_valu_probe(int32_t kind, int32_t iters, int32_t blocks, float* out, xp_stream stream);

/* Library version string. */
const char* xp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* XEPHOT_H_ */

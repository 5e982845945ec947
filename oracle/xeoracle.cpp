// xeoracle.cpp -- plain FP64 CPU reference of the optical-photon transport.
//
// TEST INFRASTRUCTURE ONLY.  This file is the oracle that the HIP path is
// checked against; only the test suite, the smoke check and the benchmark's
// CPU-baseline leg may load it.  It shares no code, header, table or constant
// generator with the HIP library: it takes the same *input arrays* (mesh,
// optical tables, sources) and computes every photon history on its own, one
// photon at a time, in double precision, with brute-force closest-hit search
// (an optional plain binary BVH gives the identical answer faster on large
// meshes; the tests check that equality).
//
// What it computes follows the paper's description of the simulated processes
// (section "Optical properties", table tab:optical, and the validation checks
// of section "Comparison of Chroma and Geant4"):
//   * isotropic emission from point sources or from points uniform in the
//     active volume (the LCE and average-LCE studies);
//   * bulk absorption with absorption length L_abs, Rayleigh scattering with
//     scattering length L_Rayleigh (exponential free paths);
//   * Rayleigh scattering with the dipole angular law that the appendix
//     (item 3) requires to match theory;
//   * surfaces whose reflectivity is given explicitly, split into diffuse and
//     specular parts and independent of the incidence angle, and Fresnel
//     reflection/refraction (with total internal reflection) only at
//     boundaries between the dielectrics quartz, LXe and GXe;
//   * specular reflection that stays defined at normal incidence (appendix
//     item 1) and a deterministic choice at the junction of two planes
//     (appendix item 2);
//   * detection at photosensors: a photon reaching the photosensitive area is
//     collected with the sensor's detection probability (the LCE definition
//     of the Z-scan check counts photons reaching that area);
//   * optionally, an emission time from the two-component exponential
//     scintillation decay (section "Optical properties": singlet and triplet
//     time constants and the singlet fraction), to which the time of flight
//     (path length times n / c per medium) is added; the arrival times of
//     detected photons give t90 (section "Light collection efficiency");
//   * optionally, a wavelength per photon from the Gaussian emission spectrum
//     (section "Optical properties": mean and FWHM), material properties
//     interpolated in wavelength, and surfaces whose reflectance follows from
//     a complex refractive index or a thin dielectric film on such a
//     substrate (the silicon backing plates and Al/MgF2 coatings of section
//     "Alternative designs").
// Where the paper is silent (random-number schedule, polarization after
// Fresnel, the self-intersection epsilon, ...) the reading used here is the
// one documented with the library's public header; each is restated at the
// function that implements it.
//
// Build: g++ -O2 -std=c++17 -fopenmp -ffp-contract=off -shared -fPIC
//
// Precision: the transport arithmetic is written in the type `real`, FP64 by
// default.  Built with -DXEORACLE_FP32 the same source computes it in FP32 (a
// diagnostic build: when the HIP path and the FP64 oracle part on a photon,
// the FP32 build shows whether single-precision rounding alone parts them
// there).  The BVH box test stays in FP64 and the gradient scores are
// evaluated in FP64 in both builds.

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <cstdio>
#include <algorithm>
#include <limits>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

#ifdef XEORACLE_FP32
using real = float;
#else
using real = double;
#endif

constexpr real kPi = real(3.14159265358979323846);
constexpr real kC = real(0.299792458);  // speed of light in vacuum, m/ns
const real kInf = std::numeric_limits<real>::infinity();
const double kInfD = std::numeric_limits<double>::infinity();

// terminal flags
enum : int32_t {
  F_ALIVE = 0, F_DETECT = 1, F_SENSOR_ABSORB = 2, F_SURFACE_ABSORB = 3, F_BULK_ABSORB = 4,
  F_ESCAPED = 5, F_MAX_STEPS = 6, F_NAN_ABORT = 7, F_GEOMETRY_ERROR = 0x100
};

// ---------------------------------------------------------------------------
// Philox-4x32-10, written from Salmon, Moraes, Dror and Shaw, "Parallel random
// numbers: as easy as 1, 2, 3" (SC'11): ten rounds of two 32x32->64 products
// with multipliers 0xD2511F53 and 0xCD9E8D57, the Weyl key bumps 0x9E3779B9 and
// 0xBB67AE85 between rounds.
// ---------------------------------------------------------------------------
struct U4 { uint32_t v[4]; };

U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1) {
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint64_t p0 = uint64_t(0xD2511F53u) * c0;
    const uint64_t p1 = uint64_t(0xCD9E8D57u) * c2;
    const uint32_t n0 = uint32_t(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n1 = uint32_t(p1);
    const uint32_t n2 = uint32_t(p0 >> 32) ^ c3 ^ k1;
    const uint32_t n3 = uint32_t(p0);
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  return U4{{c0, c1, c2, c3}};
}

// u = (top 23 bits + 1/2) / 2^23 = (2k + 1) / 2^24 with k < 2^23: strictly inside
// (0, 1) and exactly representable in FP32 as well as FP64.
double u01_exact(uint32_t x) { return (double(x >> 9) + 0.5) * (1.0 / 8388608.0); }
real u01(uint32_t x) { return real(u01_exact(x)); }

// Draw schedule (the paper names no generator): key = the 64-bit seed, counter
// = (photon id lo, photon id hi, step, sub-stream).  Step 0 is emission
// (sub 0: direction and polarization, sub 1: position for volume sources);
// step s >= 1, sub 0: free paths and the surface/Fresnel decision; sub 1:
// diffuse reflection; sub 2+j: Rayleigh trial j.
struct Draw { real u[4]; };
Draw draw(uint64_t seed, uint64_t pid, uint32_t step, uint32_t sub) {
  U4 r = philox4x32_10(uint32_t(pid), uint32_t(pid >> 32), step, sub,
                       uint32_t(seed), uint32_t(seed >> 32));
  return Draw{{u01(r.v[0]), u01(r.v[1]), u01(r.v[2]), u01(r.v[3])}};
}

// ---------------------------------------------------------------------------
// vectors
// ---------------------------------------------------------------------------
struct V3 { real x, y, z; };
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(real s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline real dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline real norm(V3 a) { return std::sqrt(dot(a, a)); }
inline V3 normalize(V3 a) { return (real(1) / norm(a)) * a; }
inline bool finite3(V3 a) { return std::isfinite(a.x) && std::isfinite(a.y) && std::isfinite(a.z); }
inline real comp(V3 a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }
inline V3 v3(const double* p) { return V3{real(p[0]), real(p[1]), real(p[2])}; }

// Orthonormal basis (b1, b2, n) for a unit n: the construction of Duff,
// Burgess, Christensen, Hery, Kensler, Liani and Villemin, "Building an
// orthonormal basis, revisited" (JCGT 2017), with its two branches (s = +1,
// valid for n_z > -1; s = -1, valid for n_z < 1) switched at n_z = -1/2 instead
// of at the sign of n_z.  Detector walls have normals in the xy plane, where
// the sign of n_z is rounding noise; the threshold keeps the basis a function
// of the geometry.
void onb(V3 n, V3& b1, V3& b2) {
  const real s = n.z >= real(-0.5) ? real(1) : real(-1);
  const real a = real(-1) / (s + n.z);
  const real b = n.x * n.y * a;
  b1 = {real(1) + s * n.x * n.x * a, s * b, -s * n.x};
  b2 = {b, s + n.y * n.y * a, -n.y};
}

// Isotropic unit vector: cos(theta) = 1 - 2 u0, phi = 2 pi u1.
V3 isotropic(real u0, real u1) {
  const real c = real(1) - real(2) * u0;
  const real s = std::sqrt(std::max(real(0), (real(1) - c) * (real(1) + c)));
  const real ph = real(2) * kPi * u1;
  return {s * std::cos(ph), s * std::sin(ph), c};
}

// Linear polarization at angle 2 pi u in the plane perpendicular to d.
V3 random_polarization(V3 d, real u) {
  V3 b1, b2;
  onb(d, b1, b2);
  const real ps = real(2) * kPi * u;
  return std::cos(ps) * b1 + std::sin(ps) * b2;
}

// ---------------------------------------------------------------------------
// scene
// ---------------------------------------------------------------------------
struct Surface {
  real p_detect, p_absorb, r_diffuse, r_specular, p_transmit;
  int32_t grad_param, flags;
  int32_t model;                 // 0 explicit partition, 1 complex index, 2 thin film
  real n_re, n_im;               // substrate index n + i k (models 1 and 2)
  real film_n, film_d_nm;        // film index and thickness (model 2)
};
struct Material { real n, abs_length, rayleigh_length; };
// one sample of a material's dispersion table
struct DispPoint { real lambda_nm, n, abs_length, rayleigh_length; };

struct BNode { double lo[3], hi[3]; int32_t left, right, first, count; };

struct Scene {
  std::vector<V3> v0, v1, v2;       // triangle vertices (copies of the float inputs)
  std::vector<int32_t> mat_in, mat_out, surf, sensor;
  std::vector<Material> mats;
  std::vector<std::vector<DispPoint>> disp;  // per material; empty: no wavelength dependence
  std::vector<Surface> surfs;
  std::vector<int32_t> channel;    // sensor -> hit-map column
  int32_t n_channels = 0;
  int32_t n_sensors = 0;
  // optional plain BVH (binary, median split); leaves index `order`
  bool use_bvh = false;
  std::vector<BNode> nodes;
  std::vector<int32_t> order;
};

// Watertight ray/triangle test of Woop, Benthin and Wald, "Watertight
// ray/triangle intersection" (JCGT 2013), in the precision `real`, edges
// inclusive, both faces.  Returns the hit distance or +inf.
struct Ray { V3 o, d; int kx, ky, kz; real sx, sy, sz; };

Ray make_ray(V3 o, V3 d) {
  Ray r{o, d, 0, 0, 0, 0, 0, 0};
  const real ax = std::fabs(d.x), ay = std::fabs(d.y), az = std::fabs(d.z);
  r.kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
  r.kx = (r.kz + 1) % 3;
  r.ky = (r.kx + 1) % 3;
  if (comp(d, r.kz) < 0) std::swap(r.kx, r.ky);
  r.sx = comp(d, r.kx) / comp(d, r.kz);
  r.sy = comp(d, r.ky) / comp(d, r.kz);
  r.sz = real(1) / comp(d, r.kz);
  return r;
}

real intersect(const Ray& r, V3 p0, V3 p1, V3 p2) {
  const V3 a = p0 - r.o, b = p1 - r.o, c = p2 - r.o;
  const real ax = comp(a, r.kx) - r.sx * comp(a, r.kz), ay = comp(a, r.ky) - r.sy * comp(a, r.kz);
  const real bx = comp(b, r.kx) - r.sx * comp(b, r.kz), by = comp(b, r.ky) - r.sy * comp(b, r.kz);
  const real cx = comp(c, r.kx) - r.sx * comp(c, r.kz), cy = comp(c, r.ky) - r.sy * comp(c, r.kz);
  const real u = cx * by - cy * bx;
  const real v = ax * cy - ay * cx;
  const real w = bx * ay - by * ax;
  if ((u < 0 || v < 0 || w < 0) && (u > 0 || v > 0 || w > 0)) return kInf;
  const real det = u + v + w;
  if (det == real(0)) return kInf;
  const real az = r.sz * comp(a, r.kz), bz = r.sz * comp(b, r.kz), cz = r.sz * comp(c, r.kz);
  const real t = (u * az + v * bz + w * cz) / det;
  return t;
}

struct Hit { int32_t tri; real t; };

// Closest hit among all triangles other than `skip` with t in (tmin, tmax];
// equal distances go to the lower triangle index.
inline void consider(const Scene& sc, const Ray& r, int32_t j, real tmin, Hit& best) {
  const real t = intersect(r, sc.v0[j], sc.v1[j], sc.v2[j]);
  if (!(t > tmin) || !(t <= best.t) || !(t < kInf)) return;  // a miss is +inf
  if (t < best.t || best.tri < 0 || j < best.tri) best = Hit{j, t};
}

Hit closest_hit_brute(const Scene& sc, V3 o, V3 d, real tmin, real tmax, int32_t skip) {
  const Ray r = make_ray(o, d);
  Hit best{-1, tmax};
  const int32_t nt = int32_t(sc.v0.size());
  for (int32_t j = 0; j < nt; ++j) {
    if (j == skip) continue;
    consider(sc, r, j, tmin, best);
  }
  return best;
}

// (in FP64 in both builds: the BVH only accelerates the search, its boxes
// are padded beyond the rounding of the triangle test)
bool box_hit(const BNode& n, const double (&oc)[3], const double (&ic)[3], double tmin, double tmax) {
  double t0 = tmin, t1 = tmax;
  for (int k = 0; k < 3; ++k) {
    double a = (n.lo[k] - oc[k]) * ic[k], b = (n.hi[k] - oc[k]) * ic[k];
    if (std::isnan(a)) a = -kInfD;  // ray parallel to the slab, origin on its face
    if (std::isnan(b)) b = kInfD;
    if (a > b) std::swap(a, b);
    t0 = std::max(t0, a);
    t1 = std::min(t1, b * (1.0 + 1e-12));
    if (t0 > t1) return false;
  }
  return true;
}

Hit closest_hit_bvh(const Scene& sc, V3 o, V3 d, real tmin, real tmax, int32_t skip) {
  const Ray r = make_ray(o, d);
  const double oc[3] = {double(o.x), double(o.y), double(o.z)};
  const double ic[3] = {1.0 / double(d.x), 1.0 / double(d.y), 1.0 / double(d.z)};
  Hit best{-1, tmax};
  int32_t stack[128];
  int sp = 0;
  stack[sp++] = 0;
  while (sp > 0) {
    const BNode& n = sc.nodes[stack[--sp]];
    if (!box_hit(n, oc, ic, 0.0, double(best.t))) continue;
    if (n.count > 0) {
      for (int32_t k = 0; k < n.count; ++k) {
        const int32_t j = sc.order[n.first + k];
        if (j != skip) consider(sc, r, j, tmin, best);
      }
    } else {
      stack[sp++] = n.left;
      stack[sp++] = n.right;
    }
  }
  return best;
}

Hit closest_hit(const Scene& sc, V3 o, V3 d, real tmin, real tmax, int32_t skip) {
  return sc.use_bvh ? closest_hit_bvh(sc, o, d, tmin, tmax, skip)
                    : closest_hit_brute(sc, o, d, tmin, tmax, skip);
}

void build_bvh(Scene& sc) {
  const int32_t nt = int32_t(sc.v0.size());
  sc.order.resize(nt);
  for (int32_t i = 0; i < nt; ++i) sc.order[i] = i;
  std::vector<V3> cen(nt);
  for (int32_t i = 0; i < nt; ++i) cen[i] = (real(1) / real(3)) * (sc.v0[i] + sc.v1[i] + sc.v2[i]);
  sc.nodes.clear();
  sc.nodes.reserve(2 * size_t(nt) + 1);
  struct Item { int32_t node, first, count; };
  std::vector<Item> work;
  sc.nodes.push_back(BNode{});
  work.push_back({0, 0, nt});
  while (!work.empty()) {
    Item it = work.back();
    work.pop_back();
    BNode n{};
    for (int k = 0; k < 3; ++k) { n.lo[k] = kInfD; n.hi[k] = -kInfD; }
    double clo[3] = {kInfD, kInfD, kInfD}, chi[3] = {-kInfD, -kInfD, -kInfD};
    for (int32_t i = it.first; i < it.first + it.count; ++i) {
      const int32_t j = sc.order[i];
      for (const V3& p : {sc.v0[j], sc.v1[j], sc.v2[j]})
        for (int k = 0; k < 3; ++k) {
          n.lo[k] = std::min(n.lo[k], double(comp(p, k)));
          n.hi[k] = std::max(n.hi[k], double(comp(p, k)));
        }
      for (int k = 0; k < 3; ++k) {
        clo[k] = std::min(clo[k], double(comp(cen[j], k)));
        chi[k] = std::max(chi[k], double(comp(cen[j], k)));
      }
    }
    // pad: a box test must never drop a triangle the triangle test hits (in
    // the FP32 build that test rounds to about 1e-7 relative)
    const double rel_pad = sizeof(real) == sizeof(double) ? 1e-9 : 1e-5;
    for (int k = 0; k < 3; ++k) {
      const double pad = rel_pad * (1.0 + std::fabs(n.lo[k]) + std::fabs(n.hi[k]));
      n.lo[k] -= pad;
      n.hi[k] += pad;
    }
    if (it.count <= 4) {
      n.left = n.right = -1;
      n.first = it.first;
      n.count = it.count;
      sc.nodes[it.node] = n;
      continue;
    }
    int axis = 0;
    for (int k = 1; k < 3; ++k)
      if (chi[k] - clo[k] > chi[axis] - clo[axis]) axis = k;
    const int32_t mid = it.first + it.count / 2;
    std::nth_element(sc.order.begin() + it.first, sc.order.begin() + mid,
                     sc.order.begin() + it.first + it.count, [&](int32_t a, int32_t b) {
                       const double ca = comp(cen[a], axis), cb = comp(cen[b], axis);
                       return ca < cb || (ca == cb && a < b);
                     });
    n.left = int32_t(sc.nodes.size());
    n.right = n.left + 1;
    n.first = 0;
    n.count = 0;
    sc.nodes[it.node] = n;
    sc.nodes.push_back(BNode{});
    sc.nodes.push_back(BNode{});
    work.push_back({n.left, it.first, mid - it.first});
    work.push_back({n.right, mid, it.first + it.count - mid});
  }
}

// ---------------------------------------------------------------------------
// photon state and interactions
// ---------------------------------------------------------------------------
struct Photon {
  V3 pos, dir, pol;
  real time;
  real wavelength;      // nm
  int32_t medium, last_tri, steps, flag, event, sensor;
  real path_len;        // path length inside the material bound to gradient params 0/1
  int32_t n_scatter;    // Rayleigh scatters in that material
  real sum_inv_r;       // sum over reflections on surfaces tagged "reflectivity" of 1/R
  real sum_inv_t;       // sum over transmissions through surfaces tagged "transparency" of 1/T
};

// Rayleigh scattering with the dipole law.  A trial direction k' is drawn
// isotropically and the new polarization is the old one projected onto the
// plane perpendicular to k'; the trial is kept with probability 1 - (e.k')^2,
// the squared length of that projection, which is the dipole emission pattern
// sin^2 of the angle to the polarization.  Averaged over e perpendicular to the
// old direction this gives (3/8)(1 + cos^2 theta) in the scattering angle.
// After 64 rejections the 64th trial is kept (probability 3^-64).
void rayleigh(Photon& p, uint64_t seed, uint64_t pid, uint32_t step) {
  V3 k{0, 0, 1}, e{1, 0, 0};
  for (uint32_t j = 0; j < 64; ++j) {
    const Draw r = draw(seed, pid, step, 2 + j);
    k = isotropic(r.u[0], r.u[1]);
    const real ek = dot(p.pol, k);
    e = p.pol - ek * k;
    if (r.u[2] < real(1) - ek * ek) break;
  }
  p.dir = k;
  p.pol = normalize(e);
}

// Lambertian (diffuse) reflection into the hemisphere of n_out:
// cos(theta) = sqrt(u0), phi = 2 pi u1; a fresh random linear polarization.
void lambertian(Photon& p, V3 n_out, const Draw& r) {
  V3 b1, b2;
  onb(n_out, b1, b2);
  const real ct = std::sqrt(r.u[0]);
  const real st = std::sqrt(std::max(real(0), real(1) - r.u[0]));
  const real ph = real(2) * kPi * r.u[1];
  p.dir = normalize(st * std::cos(ph) * b1 + st * std::sin(ph) * b2 + ct * n_out);
  p.pol = random_polarization(p.dir, r.u[2]);
}

// Mirror reflection about the plane with unit normal n (either orientation):
// d' = d - 2 (d.n) n and the same for the polarization.  Defined at normal
// incidence, where it returns -d (appendix item 1).
void specular(Photon& p, V3 n) {
  p.dir = normalize(p.dir - (real(2) * dot(p.dir, n)) * n);
  p.pol = normalize(p.pol - (real(2) * dot(p.pol, n)) * n);
}

// Fresnel reflection / refraction at a boundary between real refractive
// indices n1 (incident side) and n2, for a linearly polarized photon.
// nhat is the unit normal pointing back into the incident medium.  The
// polarization is split into s (perpendicular to the plane of incidence) and
// p parts; amplitude coefficients r_s, r_p, t_s, t_p in the Born & Wolf
// convention; the reflection probability is R = a_s^2 r_s^2 + a_p^2 r_p^2.
// At normal incidence the plane of incidence is undefined and s is taken
// along the polarization itself.  Above the critical angle the photon is
// totally reflected.  Returns true if it was transmitted.
bool fresnel(Photon& p, V3 nhat, real n1, real n2, real u) {
  const V3 d = p.dir, e = p.pol;
  const real ci = -dot(d, nhat);
  const real eta = n1 / n2;
  const real st2 = eta * eta * (real(1) - ci * ci);
  if (st2 >= real(1)) {  // total internal reflection
    specular(p, nhat);
    return false;
  }
  const real ct = std::sqrt(real(1) - st2);
  const real rs = (n1 * ci - n2 * ct) / (n1 * ci + n2 * ct);
  const real rp = (n2 * ci - n1 * ct) / (n2 * ci + n1 * ct);
  const real ts = real(2) * n1 * ci / (n1 * ci + n2 * ct);
  const real tp = real(2) * n1 * ci / (n2 * ci + n1 * ct);
  V3 sv = cross(d, nhat);
  const real sl = norm(sv);
  V3 s = (sl < real(1e-6)) ? e : (real(1) / sl) * sv;
  const real as = dot(e, s);
  const real ap = dot(e, cross(s, d));
  const real R = as * as * rs * rs + ap * ap * rp * rp;
  if (u < R) {
    const V3 dr = normalize(d + (real(2) * ci) * nhat);
    p.pol = normalize((rs * as) * s + (rp * ap) * cross(s, dr));
    p.dir = dr;
    return false;
  }
  const V3 dt = normalize(eta * d + (eta * ci - ct) * nhat);
  p.pol = normalize((ts * as) * s + (tp * ap) * cross(s, dt));
  p.dir = dt;
  return true;
}

// ---------------------------------------------------------------------------
// wavelength dependence
// ---------------------------------------------------------------------------

// Material properties at wavelength lambda from its dispersion table: the
// refractive index and the attenuation coefficients 1/L (so that an infinite
// length is a zero coefficient) are interpolated linearly between the two
// neighbouring samples and held constant beyond the first and last.
Material material_at(const Scene& sc, int32_t m, real lambda) {
  const std::vector<DispPoint>& t = sc.disp[m];
  if (t.empty()) return sc.mats[m];
  auto inv = [](real L) { return std::isinf(L) ? real(0) : real(1) / L; };
  auto len = [](real mu) { return mu > real(0) ? real(1) / mu : kInf; };
  if (lambda <= t.front().lambda_nm)
    return Material{t.front().n, t.front().abs_length, t.front().rayleigh_length};
  if (lambda >= t.back().lambda_nm)
    return Material{t.back().n, t.back().abs_length, t.back().rayleigh_length};
  size_t i = 0;
  while (t[i + 1].lambda_nm < lambda) ++i;
  const DispPoint& a = t[i];
  const DispPoint& b = t[i + 1];
  const real w = (lambda - a.lambda_nm) / (b.lambda_nm - a.lambda_nm);
  return Material{a.n + w * (b.n - a.n),
                  len(inv(a.abs_length) + w * (inv(b.abs_length) - inv(a.abs_length))),
                  len(inv(a.rayleigh_length) + w * (inv(b.rayleigh_length) - inv(a.rayleigh_length)))};
}

using C = std::complex<real>;

// Amplitude reflection coefficients (s, p) for light arriving from a medium of
// real index n1 at incidence cosine ci on (model 1) a medium of complex index
// n2 = n + i k, or (model 2) a film of real index nf and thickness d on that
// medium, at vacuum wavelength lambda.  With q_j = sqrt(n_j^2 - n1^2 sin^2)
// (= n_j cos(theta_j), principal branch, so waves decay into absorbing or
// evanescent layers), the interface coefficients are
//   r_s = (q_a - q_b) / (q_a + q_b),  r_p = (n_b^2 q_a - n_a^2 q_b) / (n_b^2 q_a + n_a^2 q_b)
// (the Born & Wolf convention of the dielectric case), and a film combines
// its two interfaces with the phase beta = 2 pi d q_f / lambda:
//   r = (r_01 + r_12 e^{2 i beta}) / (1 + r_01 r_12 e^{2 i beta}).
void film_reflection(int32_t model, real n1, real ci, real n_re, real n_im, real nf,
                     real d_nm, real lambda, C& rs, C& rp) {
  const C n2(n_re, n_im);
  const real s2 = n1 * n1 * (real(1) - ci * ci);  // n1^2 sin^2(theta_i)
  const C q1(n1 * ci, real(0));
  const C q2 = std::sqrt(n2 * n2 - s2);
  const C e1(n1 * n1, real(0)), e2 = n2 * n2;
  if (model == 1) {
    rs = (q1 - q2) / (q1 + q2);
    rp = (e2 * q1 - e1 * q2) / (e2 * q1 + e1 * q2);
    return;
  }
  const C ef(nf * nf, real(0));
  const C qf = std::sqrt(ef - s2);
  const C r01s = (q1 - qf) / (q1 + qf), r12s = (qf - q2) / (qf + q2);
  const C r01p = (ef * q1 - e1 * qf) / (ef * q1 + e1 * qf);
  const C r12p = (e2 * qf - ef * q2) / (e2 * qf + ef * q2);
  const C ph = std::exp(C(real(0), real(2)) * (real(2) * kPi * d_nm / lambda) * qf);
  rs = (r01s + r12s * ph) / (real(1) + r01s * r12s * ph);
  rp = (r01p + r12p * ph) / (real(1) + r01p * r12p * ph);
}

// Reflection off a surface of model 1 or 2: the photon is reflected
// specularly with probability R = a_s^2 |r_s|^2 + a_p^2 |r_p|^2 (a_s, a_p:
// components of its linear polarization along s and p; at normal incidence s
// is taken along the polarization).  The reflected photon stays linearly
// polarized, its s and p components scaled by |r| with the sign of Re r (the
// real, dielectric limit).  Returns true if reflected.
bool model_reflection(Photon& p, V3 nhat, real n1, const Surface& s, real u) {
  const V3 d = p.dir, e = p.pol;
  const real ci = -dot(d, nhat);
  C rs, rp;
  film_reflection(s.model, n1, ci, s.n_re, s.n_im, s.film_n, s.film_d_nm, p.wavelength, rs, rp);
  V3 sv = cross(d, nhat);
  const real sl = norm(sv);
  const V3 sd = (sl < real(1e-6)) ? e : (real(1) / sl) * sv;
  const real as = dot(e, sd);
  const real ap = dot(e, cross(sd, d));
  const real Rs = std::norm(rs), Rp = std::norm(rp);
  const real R = as * as * Rs + ap * ap * Rp;
  if (!(u < R)) return false;
  const V3 dr = normalize(d + (real(2) * ci) * nhat);
  const real ms = std::copysign(std::abs(rs), rs.real());
  const real mp = std::copysign(std::abs(rp), rp.real());
  p.pol = normalize((ms * as) * sd + (mp * ap) * cross(sd, dr));
  p.dir = dr;
  return true;
}

// ---------------------------------------------------------------------------
// sources
// ---------------------------------------------------------------------------
struct Sources {
  int32_t kind;            // 0 points, 1 uniform cylinder, 2 explicit
  int32_t medium;
  int64_t n_photons;
  int64_t n_sources;
  const float* positions;
  const int64_t* offsets;  // may be null: count_per_source photons each
  int64_t count_per_source;
  int32_t per_source_events;
  const float* directions;
  const float* polarizations;
  real cyl_radius, cyl_zlo, cyl_zhi;
  int32_t time_profile;    // 0: t = 0 at emission; 1: scintillation decay
  real tau_singlet, tau_triplet, singlet_fraction;
  real wavelength_nm, wavelength_fwhm_nm;  // Gaussian spectrum (FWHM 0: one line)
};

// Wavelength from the Gaussian emission spectrum: Philox block (step 0,
// sub 3), Box-Muller with sigma = FWHM / (2 sqrt(2 ln 2)).
real emission_wavelength(uint64_t seed, uint64_t pid, real mean, real fwhm) {
  if (!(fwhm > real(0))) return mean;
  const Draw r = draw(seed, pid, 0, 3);
  const real sigma = real(double(fwhm) / (2.0 * std::sqrt(2.0 * std::log(2.0))));
  return mean + sigma * std::sqrt(real(-2) * std::log(r.u[0])) * std::cos(real(2) * kPi * r.u[1]);
}

// Scintillation emission time: the photon comes from the singlet state with
// probability singlet_fraction (u0 of Philox block (step 0, sub 2)), else from
// the triplet state, and is emitted after an exponential delay with that
// state's time constant (inverse CDF: t = -tau ln u1).
real scintillation_time(uint64_t seed, uint64_t pid, real tau_singlet, real tau_triplet,
                        real singlet_fraction, bool& singlet);

int64_t source_of(const Sources& s, int64_t i) {
  if (s.offsets == nullptr) return i / s.count_per_source;
  // last source whose offset is <= i (sources with zero photons are skipped)
  int64_t lo = 0, hi = s.n_sources;  // offsets[lo] <= i < offsets[hi]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) / 2;
    if (s.offsets[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

// Emission of photon i (launch-local index) with id pid: position from the
// source, isotropic direction, random linear polarization, t = 0.
void emit(Photon& p, const Sources& s, int64_t i, uint64_t seed, uint64_t pid) {
  p.time = 0;
  p.medium = s.medium;
  p.last_tri = -1;
  p.steps = 0;
  p.flag = F_ALIVE;
  p.event = 0;
  p.sensor = -1;
  p.path_len = 0;
  p.n_scatter = 0;
  p.sum_inv_r = 0;
  p.sum_inv_t = 0;
  if (s.kind == 2) {
    p.pos = {real(s.positions[3 * i]), real(s.positions[3 * i + 1]), real(s.positions[3 * i + 2])};
    p.dir = normalize(V3{real(s.directions[3 * i]), real(s.directions[3 * i + 1]),
                         real(s.directions[3 * i + 2])});
    p.pol = V3{real(s.polarizations[3 * i]), real(s.polarizations[3 * i + 1]),
               real(s.polarizations[3 * i + 2])};
    p.pol = normalize(p.pol - dot(p.pol, p.dir) * p.dir);
    return;
  }
  const Draw r = draw(seed, pid, 0, 0);
  p.dir = isotropic(r.u[0], r.u[1]);
  p.pol = random_polarization(p.dir, r.u[2]);
  if (s.kind == 0) {
    const int64_t src = source_of(s, i);
    p.pos = {real(s.positions[3 * src]), real(s.positions[3 * src + 1]), real(s.positions[3 * src + 2])};
    p.event = s.per_source_events ? int32_t(src) : 0;
  } else {
    // uniform in the cylinder r <= R, z_lo <= z <= z_hi: r = R sqrt(u0), phi = 2 pi u1
    const Draw q = draw(seed, pid, 0, 1);
    const real rr = s.cyl_radius * std::sqrt(q.u[0]);
    const real ph = real(2) * kPi * q.u[1];
    p.pos = {rr * std::cos(ph), rr * std::sin(ph), s.cyl_zlo + (s.cyl_zhi - s.cyl_zlo) * q.u[2]};
  }
}

real scintillation_time(uint64_t seed, uint64_t pid, real tau_singlet, real tau_triplet,
                        real singlet_fraction, bool& singlet) {
  const Draw r = draw(seed, pid, 0, 2);
  singlet = r.u[0] < singlet_fraction;
  return -(singlet ? tau_singlet : tau_triplet) * std::log(r.u[1]);
}

// Emission plus the emission time of the source's time profile.
void emit_timed(Photon& p, const Sources& s, int64_t i, uint64_t seed, uint64_t pid) {
  emit(p, s, i, seed, pid);
  p.wavelength = emission_wavelength(seed, pid, s.wavelength_nm, s.wavelength_fwhm_nm);
  if (s.time_profile == 1) {
    bool singlet;
    p.time = scintillation_time(seed, pid, s.tau_singlet, s.tau_triplet, s.singlet_fraction, singlet);
  }
}

// eps: hits on triangles other than the last one count for t > eps.
// surface_offset: after a (non-terminal) surface interaction the photon
// restarts this far from the surface, along the normal on the side it leaves
// toward.  This keeps a photon that lands near the shared edge of two coplanar
// triangles from re-hitting the neighbour at t ~ 0 from the wrong side, while
// a neighbouring face of a concave corner still lies ahead of it (a window of
// t values below eps would let such a photon pass through that face).
struct Params {
  uint64_t seed;
  uint64_t pid_base;
  int32_t max_steps;
  real eps;
  int32_t grad_material;
  real surface_offset;
};

inline real free_path(real length, real u) {
  return std::isinf(length) ? kInf : -length * std::log(u);
}

// Transport of one photon until it ends in exactly one terminal state.
void transport(const Scene& sc, const Params& prm, uint64_t pid, Photon& p) {
  for (int32_t step = 1; step <= prm.max_steps; ++step) {
    p.steps = step;
    const Material m = material_at(sc, p.medium, p.wavelength);
    const Draw r = draw(prm.seed, pid, uint32_t(step), 0);
    const real d_abs = free_path(m.abs_length, r.u[0]);
    const real d_sca = free_path(m.rayleigh_length, r.u[1]);
    const real d_bulk = std::min(d_abs, d_sca);
    const Hit h = closest_hit(sc, p.pos, p.dir, prm.eps, d_bulk, p.last_tri);
    if (h.tri < 0) {
      if (std::isinf(d_bulk)) { p.flag |= F_ESCAPED; return; }
      p.pos = p.pos + d_bulk * p.dir;
      p.time += d_bulk * m.n / kC;
      if (p.medium == prm.grad_material) p.path_len += d_bulk;
      if (d_abs <= d_sca) { p.flag |= F_BULK_ABSORB; return; }
      if (p.medium == prm.grad_material) p.n_scatter += 1;
      rayleigh(p, prm.seed, pid, uint32_t(step));
      p.last_tri = -1;
    } else {
      const int32_t k = h.tri;
      p.pos = p.pos + h.t * p.dir;
      p.time += h.t * m.n / kC;
      if (p.medium == prm.grad_material) p.path_len += h.t;
      const V3 N = normalize(cross(sc.v1[k] - sc.v0[k], sc.v2[k] - sc.v0[k]));
      const bool from_outer = dot(p.dir, N) < real(0);
      const int32_t m_from = from_outer ? sc.mat_out[k] : sc.mat_in[k];
      const int32_t m_to = from_outer ? sc.mat_in[k] : sc.mat_out[k];
      if (m_from != p.medium) { p.flag |= F_GEOMETRY_ERROR; p.medium = m_from; }
      const V3 n_back = from_outer ? N : real(-1) * N;  // unit normal on the arrival side
      const int32_t si = sc.surf[k];
      if (si >= 0) {
        const Surface& s = sc.surfs[si];
        const bool is_sensor = sc.sensor[k] >= 0;
        if ((s.flags & 1) && !from_outer) {  // back of a front-only sensor: absorber
          p.flag |= F_SURFACE_ABSORB;
          p.last_tri = k;
          return;
        }
        const real u = r.u[2];
        if (s.model != 0) {
          // reflectance from the complex index / film; the rest enters the
          // surface's material: detected on a sensor, absorbed elsewhere
          if (model_reflection(p, n_back, material_at(sc, m_from, p.wavelength).n, s, u)) {
            p.pos = p.pos + prm.surface_offset * n_back;
            p.last_tri = k;
            if (!finite3(p.pos) || !finite3(p.dir) || !finite3(p.pol)) { p.flag |= F_NAN_ABORT; return; }
            continue;
          }
          if (is_sensor) { p.flag |= F_DETECT; p.sensor = sc.sensor[k]; }
          else p.flag |= F_SURFACE_ABSORB;
          p.last_tri = k;
          return;
        }
        real c = s.p_detect;
        if (u < c) {
          if (is_sensor) { p.flag |= F_DETECT; p.sensor = sc.sensor[k]; }
          else p.flag |= F_SURFACE_ABSORB;
          p.last_tri = k;
          return;
        }
        c += s.p_absorb;
        if (u < c) {
          if (is_sensor) { p.flag |= F_SENSOR_ABSORB; p.sensor = sc.sensor[k]; }
          else p.flag |= F_SURFACE_ABSORB;
          p.last_tri = k;
          return;
        }
        const real r_tot = s.r_diffuse + s.r_specular;
        c += s.r_diffuse;
        bool through = false;
        if (u < c) {
          lambertian(p, n_back, draw(prm.seed, pid, uint32_t(step), 1));
          if (s.grad_param == 2) p.sum_inv_r += real(1) / r_tot;
        } else if (u < c + s.r_specular) {
          specular(p, N);
          if (s.grad_param == 2) p.sum_inv_r += real(1) / r_tot;
        } else if (s.p_transmit > real(0)) {
          p.medium = m_to;
          through = true;
          if (s.grad_param == 3) p.sum_inv_t += real(1) / s.p_transmit;
        } else {  // probabilities summing to just under one: the remainder absorbs
          p.flag |= (is_sensor ? F_SENSOR_ABSORB : F_SURFACE_ABSORB);
          if (is_sensor) p.sensor = sc.sensor[k];
          p.last_tri = k;
          return;
        }
        p.pos = p.pos + (through ? -prm.surface_offset : prm.surface_offset) * n_back;
      } else {
        const real n1 = material_at(sc, m_from, p.wavelength).n;
        const real n2 = material_at(sc, m_to, p.wavelength).n;
        bool through = true;
        if (n1 != n2) through = fresnel(p, n_back, n1, n2, r.u[2]);
        if (through) p.medium = m_to;
        p.pos = p.pos + (through ? -prm.surface_offset : prm.surface_offset) * n_back;
      }
      p.last_tri = k;
    }
    if (!finite3(p.pos) || !finite3(p.dir) || !finite3(p.pol)) { p.flag |= F_NAN_ABORT; return; }
  }
  p.flag |= F_MAX_STEPS;
}

}  // namespace

// ---------------------------------------------------------------------------
// C interface used by the tests (ctypes)
// ---------------------------------------------------------------------------
extern "C" {

struct OracleRecord {  // one per photon
  int32_t flag, last_tri, sensor, steps;
  int32_t event, medium, n_scatter, pad;
  double pos[3], dir[3], pol[3];
  double time, path_len, sum_inv_r, sum_inv_t;
  double wavelength;
};

void* oracle_scene_create(const float* vtx, int64_t nv, const int32_t* tri, int64_t nt,
                          const int32_t* mat_in, const int32_t* mat_out, const int32_t* surf,
                          const int32_t* sensor, const float* mats, int32_t n_mats,
                          const float* surf_p, const int32_t* surf_tags,
                          const float* surf_optics, int32_t n_surfs,
                          const int32_t* channel_of_sensor, int32_t n_sensors, int32_t n_channels,
                          int32_t use_bvh) {
  Scene* sc = new Scene();
  sc->v0.resize(nt); sc->v1.resize(nt); sc->v2.resize(nt);
  for (int64_t i = 0; i < nt; ++i) {
    const int32_t* t = tri + 3 * i;
    auto V = [&](int32_t j) { return V3{real(vtx[3 * j]), real(vtx[3 * j + 1]), real(vtx[3 * j + 2])}; };
    sc->v0[i] = V(t[0]); sc->v1[i] = V(t[1]); sc->v2[i] = V(t[2]);
  }
  (void)nv;
  sc->mat_in.assign(mat_in, mat_in + nt);
  sc->mat_out.assign(mat_out, mat_out + nt);
  sc->surf.assign(surf, surf + nt);
  sc->sensor.assign(sensor, sensor + nt);
  for (int32_t i = 0; i < n_mats; ++i)
    sc->mats.push_back(Material{real(mats[3 * i]), real(mats[3 * i + 1]), real(mats[3 * i + 2])});
  sc->disp.assign(sc->mats.size(), {});
  for (int32_t i = 0; i < n_surfs; ++i) {
    const float* q = surf_p + 5 * i;
    const float* o = surf_optics + 4 * i;
    sc->surfs.push_back(Surface{real(q[0]), real(q[1]), real(q[2]), real(q[3]), real(q[4]),
                                surf_tags[3 * i], surf_tags[3 * i + 1], surf_tags[3 * i + 2],
                                real(o[0]), real(o[1]), real(o[2]), real(o[3])});
  }
  sc->n_sensors = n_sensors;
  sc->n_channels = n_channels;
  sc->channel.resize(n_sensors);
  for (int32_t i = 0; i < n_sensors; ++i) sc->channel[i] = channel_of_sensor ? channel_of_sensor[i] : i;
  sc->use_bvh = use_bvh != 0;
  if (sc->use_bvh) build_bvh(*sc);
  return sc;
}

void oracle_scene_destroy(void* s) { delete static_cast<Scene*>(s); }

// Dispersion table of material m: n samples (lambda ascending); n = 0 removes it.
void oracle_scene_set_dispersion(void* scene, int32_t m, int32_t n, const float* lambda_nm,
                                 const float* index, const float* abs_length,
                                 const float* rayleigh_length) {
  Scene& sc = *static_cast<Scene*>(scene);
  sc.disp[m].clear();
  for (int32_t i = 0; i < n; ++i)
    sc.disp[m].push_back(DispPoint{real(lambda_nm[i]), real(index[i]), real(abs_length[i]),
                                   real(rayleigh_length[i])});
}

// Propagate photons with launch-local indices [i_begin, i_end) (photon id =
// pid_base + i).  Optional outputs: one record per photon (indexed i - i_begin),
// the hit map [event][channel] (int64, accumulated) and the gradient tallies
// [event][channel][4] (accumulated).  Returns 0.
int oracle_run(void* scene, int32_t kind, int32_t medium, int64_t n_photons, int64_t n_sources,
               const float* positions, const int64_t* offsets, int64_t count_per_source,
               int32_t per_source_events, const float* directions, const float* polarizations,
               double cyl_radius, double cyl_zlo, double cyl_zhi, int32_t time_profile,
               double tau_singlet, double tau_triplet, double singlet_fraction,
               double wavelength_nm, double wavelength_fwhm_nm, uint64_t seed,
               uint64_t pid_base, int32_t max_steps, double eps, int32_t grad_material,
               double surface_offset, int64_t i_begin, int64_t i_end, OracleRecord* records,
               int64_t* hit_map, double* grad, int32_t n_threads) {
  const Scene& sc = *static_cast<Scene*>(scene);
  Sources s{kind, medium, n_photons, n_sources, positions, offsets, count_per_source,
            per_source_events, directions, polarizations, real(cyl_radius), real(cyl_zlo),
            real(cyl_zhi), time_profile, real(tau_singlet), real(tau_triplet),
            real(singlet_fraction), real(wavelength_nm), real(wavelength_fwhm_nm)};
  Params prm{seed, pid_base, max_steps, real(eps), grad_material, real(surface_offset)};
  const Material& gm = sc.mats[grad_material >= 0 ? grad_material : 0];
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 256)
#endif
  for (int64_t i = i_begin; i < i_end; ++i) {
    const uint64_t pid = pid_base + uint64_t(i);
    Photon p{};
    emit_timed(p, s, i, seed, pid);
    transport(sc, prm, pid, p);
    if (records) {
      OracleRecord& rec = records[i - i_begin];
      rec.flag = p.flag; rec.last_tri = p.last_tri; rec.sensor = p.sensor; rec.steps = p.steps;
      rec.event = p.event; rec.medium = p.medium; rec.n_scatter = p.n_scatter; rec.pad = 0;
      rec.pos[0] = p.pos.x; rec.pos[1] = p.pos.y; rec.pos[2] = p.pos.z;
      rec.dir[0] = p.dir.x; rec.dir[1] = p.dir.y; rec.dir[2] = p.dir.z;
      rec.pol[0] = p.pol.x; rec.pol[1] = p.pol.y; rec.pol[2] = p.pol.z;
      rec.time = p.time; rec.path_len = p.path_len; rec.sum_inv_r = p.sum_inv_r; rec.sum_inv_t = p.sum_inv_t;
      rec.wavelength = p.wavelength;
    }
    if ((p.flag & 0xff) == F_DETECT) {
      const int64_t cell = int64_t(p.event) * sc.n_channels + sc.channel[p.sensor];
      if (hit_map) {
#ifdef _OPENMP
#pragma omp atomic
#endif
        hit_map[cell] += 1;
      }
      if (grad) {
        // score-function (likelihood-ratio) weights of a detected path:
        // d log P / d L_abs = L / L_abs^2, d log P / d L_R = L / L_R^2 - N_sca / L_R,
        // d log P / d R = (reflections) / R, d log P / d T = (transmissions) / T.
        const double L = double(p.path_len), la = double(gm.abs_length);
        const double lr = double(gm.rayleigh_length);
        const double sc0 = L / (la * la);
        const double sc1 = L / (lr * lr) - double(p.n_scatter) / lr;
        const double g[4] = {std::isfinite(sc0) ? sc0 : 0.0, std::isfinite(sc1) ? sc1 : 0.0,
                             double(p.sum_inv_r), double(p.sum_inv_t)};
        for (int q = 0; q < 4; ++q) {
#ifdef _OPENMP
#pragma omp atomic
#endif
          grad[cell * 4 + q] += g[q];
        }
      }
    }
  }
  return 0;
}

// ---- hooks for the sampler and boundary tests ----
void oracle_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  U4 r = philox4x32_10(ctr[0], ctr[1], ctr[2], ctr[3], key[0], key[1]);
  for (int k = 0; k < 4; ++k) out[k] = r.v[k];
}

double oracle_u01(uint32_t x) { return double(u01(x)); }

// 1 in the FP32 diagnostic build, 0 in the FP64 oracle.
int32_t oracle_is_fp32(void) { return sizeof(real) == sizeof(float) ? 1 : 0; }

// Emission wavelengths of photon ids pid0 .. pid0+n-1.
void oracle_wavelength(uint64_t seed, uint64_t pid0, int64_t n, double mean, double fwhm,
                       double* out) {
  for (int64_t i = 0; i < n; ++i)
    out[i] = double(emission_wavelength(seed, pid0 + uint64_t(i), real(mean), real(fwhm)));
}

// Power reflectances |r_s|^2, |r_p|^2 of a model-1/2 surface for n incidence
// cosines (from a medium of index n1, vacuum wavelength lambda).
void oracle_surface_reflectance(int32_t model, double n1, double n_re, double n_im, double film_n,
                                double film_d_nm, double lambda, int64_t n, const double* cos_i,
                                double* out_rs, double* out_rp) {
  for (int64_t i = 0; i < n; ++i) {
    C rs, rp;
    film_reflection(model, real(n1), real(cos_i[i]), real(n_re), real(n_im), real(film_n),
                    real(film_d_nm), real(lambda), rs, rp);
    out_rs[i] = double(std::norm(rs));
    out_rp[i] = double(std::norm(rp));
  }
}

// Material properties at wavelengths lambda[0..n) (index, absorption and
// Rayleigh lengths into out[3 i .. 3 i + 2]).
void oracle_material_at(void* scene, int32_t m, int64_t n, const double* lambda, double* out) {
  const Scene& sc = *static_cast<Scene*>(scene);
  for (int64_t i = 0; i < n; ++i) {
    const Material q = material_at(sc, m, real(lambda[i]));
    out[3 * i] = double(q.n);
    out[3 * i + 1] = double(q.abs_length);
    out[3 * i + 2] = double(q.rayleigh_length);
  }
}

// Scintillation emission times of photon ids pid0 .. pid0+n-1 and their state
// (1 singlet, 0 triplet).
void oracle_emission_time(uint64_t seed, uint64_t pid0, int64_t n, double tau_singlet,
                          double tau_triplet, double singlet_fraction, double* out_t,
                          int32_t* out_singlet) {
  for (int64_t i = 0; i < n; ++i) {
    bool singlet;
    out_t[i] = double(scintillation_time(seed, pid0 + uint64_t(i), real(tau_singlet),
                                         real(tau_triplet), real(singlet_fraction), singlet));
    out_singlet[i] = singlet ? 1 : 0;
  }
}

// kind 0: emission direction+polarization (step 0); kind 1: Lambertian about
// in_dir (used as the normal), sub 1 of step 1; kind 2: Rayleigh from
// (in_dir, in_pol) at step 1; kind 3: uniform-cylinder positions (out_dir holds
// the position).  Photon ids pid0 .. pid0+n-1.
void oracle_sample(int32_t kind, uint64_t seed, uint64_t pid0, int64_t n, const double* in_dir,
                   const double* in_pol, double cyl_r, double zlo, double zhi, double* out_dir,
                   double* out_pol) {
  for (int64_t i = 0; i < n; ++i) {
    const uint64_t pid = pid0 + uint64_t(i);
    Photon p{};
    if (kind == 0) {
      const Draw r = draw(seed, pid, 0, 0);
      p.dir = isotropic(r.u[0], r.u[1]);
      p.pol = random_polarization(p.dir, r.u[2]);
    } else if (kind == 1) {
      lambertian(p, v3(in_dir + 3 * i), draw(seed, pid, 1, 1));
    } else if (kind == 2) {
      p.dir = v3(in_dir + 3 * i);
      p.pol = v3(in_pol + 3 * i);
      rayleigh(p, seed, pid, 1);
    } else {
      Sources s{};
      s.kind = 1; s.cyl_radius = real(cyl_r); s.cyl_zlo = real(zlo); s.cyl_zhi = real(zhi);
      emit(p, s, int64_t(i), seed, pid);
      p.dir = p.pos;
      p.pol = V3{real(0), real(0), real(0)};
    }
    out_dir[3 * i] = p.dir.x; out_dir[3 * i + 1] = p.dir.y; out_dir[3 * i + 2] = p.dir.z;
    out_pol[3 * i] = p.pol.x; out_pol[3 * i + 1] = p.pol.y; out_pol[3 * i + 2] = p.pol.z;
  }
}

// One boundary event: Fresnel (mode 0) or explicit specular (mode 1) for a
// photon (dir, pol) meeting a plane with unit normal n (any orientation).
// Returns 1 if transmitted.
int32_t oracle_boundary(int32_t mode, const double* dir, const double* pol, const double* n,
                        double n1, double n2, double u, double* out_dir, double* out_pol) {
  Photon p{};
  p.dir = v3(dir);
  p.pol = v3(pol);
  const V3 N = v3(n);
  const V3 nb = dot(p.dir, N) < real(0) ? N : real(-1) * N;
  int32_t tr = 0;
  if (mode == 0) tr = fresnel(p, nb, real(n1), real(n2), real(u)) ? 1 : 0;
  else specular(p, N);
  out_dir[0] = p.dir.x; out_dir[1] = p.dir.y; out_dir[2] = p.dir.z;
  out_pol[0] = p.pol.x; out_pol[1] = p.pol.y; out_pol[2] = p.pol.z;
  return tr;
}

// One reflection off a complex-index (model 1) or thin-film (model 2) surface
// for a photon (dir, pol) meeting a plane with unit normal n (any
// orientation) from a medium of index n1 at wavelength lambda.  Returns 1 if
// the photon was reflected (u < R), 0 if it entered the surface.
int32_t oracle_model_boundary(int32_t model, const double* dir, const double* pol, const double* n,
                              double n1, double n_re, double n_im, double film_n, double film_d_nm,
                              double lambda, double u, double* out_dir, double* out_pol) {
  Photon p{};
  p.dir = v3(dir);
  p.pol = v3(pol);
  p.wavelength = real(lambda);
  const V3 N = v3(n);
  const V3 nb = dot(p.dir, N) < real(0) ? N : real(-1) * N;
  Surface s{};
  s.model = model;
  s.n_re = real(n_re);
  s.n_im = real(n_im);
  s.film_n = real(film_n);
  s.film_d_nm = real(film_d_nm);
  const bool refl = model_reflection(p, nb, real(n1), s, real(u));
  out_dir[0] = p.dir.x; out_dir[1] = p.dir.y; out_dir[2] = p.dir.z;
  out_pol[0] = p.pol.x; out_pol[1] = p.pol.y; out_pol[2] = p.pol.z;
  return refl ? 1 : 0;
}

// Closest hit for a batch of rays (brute force or the scene's BVH).
void oracle_closest_hit(void* scene, int64_t n, const double* orig, const double* dir, double tmin,
                        double tmax, const int32_t* skip, int32_t force_brute, int32_t* out_tri,
                        double* out_t) {
  const Scene& sc = *static_cast<Scene*>(scene);
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64)
#endif
  for (int64_t i = 0; i < n; ++i) {
    const V3 o = v3(orig + 3 * i);
    const V3 d = v3(dir + 3 * i);
    const int32_t sk = skip ? skip[i] : -1;
    const Hit h = force_brute ? closest_hit_brute(sc, o, d, real(tmin), real(tmax), sk)
                              : closest_hit(sc, o, d, real(tmin), real(tmax), sk);
    out_tri[i] = h.tri;
    out_t[i] = h.tri >= 0 ? double(h.t) : kInfD;
  }
}

int32_t oracle_max_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"

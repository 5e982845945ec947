// transport.h -- device code of the optical-photon transport (gfx950): the
// per-photon physics, the BVH traversal and the persistent transport kernel
// template.  Included by propagate.hip (forward, backward, records and
// counter variants, plus the test-hook kernels) and propagate_tally.hip (the
// variants with per-workgroup LDS tallies), each of which instantiates only
// its own kernels: keeping the instantiations apart keeps the code generated
// for each one independent of the others.
//
// One lane carries one photon.  A workgroup stages the top levels of the
// 4-wide BVH in LDS, then loops persistently: lanes whose photon has ended
// are refilled from a per-wave pool of photon ids (one wave ballot, one
// atomic per `chunk` photons), and every live lane advances its photon by one
// step: free paths for absorption and Rayleigh scattering, closest hit along
// the ray, then the bulk or surface interaction.  Photon i's random numbers
// come from Philox-4x32-10 keyed by the seed with the photon id in the
// counter, so results do not depend on which lane or wave runs the photon.
//
// The processes follow the paper's optical model (section "Optical
// properties", table tab:optical): absorption and Rayleigh scattering with
// exponential free paths; Rayleigh scattering with the dipole law (appendix
// item 3); explicit angle-independent surfaces (detect / absorb / diffuse /
// specular / transmit); Fresnel reflection and refraction with total internal
// reflection at dielectric boundaries (quartz, LXe, GXe); detection at sensors.
// Optionally: emission times from the scintillation decay, wavelengths from
// the Gaussian emission spectrum with interpolated material properties, and
// surfaces whose reflectance follows from a complex index or a thin film
// (section "Alternative designs").
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "xp_internal.h"

namespace xp {
namespace {

constexpr float kInfF = __builtin_huge_valf();
constexpr float kCns = 0.299792458f;  // m/ns

// ---------------------------------------------------------------------------
// random numbers: Philox-4x32-10 (Salmon et al., SC'11)
// ---------------------------------------------------------------------------
struct R4 { float u0, u1, u2, u3; };

// The key (the seed) must be the same in every lane of the wave: it is held in
// scalar registers.  The empty asm makes the compiler derive the round keys
// per call on the scalar unit instead of keeping all twenty live through the
// transport loop, where they crowd out other scalar values.
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
  asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    // one 32 x 32 -> 64-bit multiply-add instruction per product, and one
    // three-input bitwise instruction (truth table 0x96: a ^ b ^ c) per
    // new word
    const uint64_t p0 = uint64_t(c0) * 0xD2511F53ull;
    const uint64_t p1 = uint64_t(c2) * 0xCD9E8D57ull;
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32(uint32_t(p1 >> 32), c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32(uint32_t(p0 >> 32), c3, k1, 0x96);
    c0 = n0;
    c1 = uint32_t(p1);
    c2 = n2;
    c3 = uint32_t(p0);
  }
  return make_uint4(c0, c1, c2, c3);
}

// (2k + 1) / 2^24 from the top 23 bits: exact in FP32, strictly inside (0, 1)
__device__ __forceinline__ float u01(uint32_t x) {
  return (float(x >> 9) + 0.5f) * 1.1920928955078125e-7f;
}

__device__ __forceinline__ R4 draw(uint32_t seed_lo, uint32_t seed_hi, uint64_t pid, uint32_t step,
                                   uint32_t sub) {
  const uint4 r = philox(uint32_t(pid), uint32_t(pid >> 32), step, sub, seed_lo, seed_hi);
  return R4{u01(r.x), u01(r.y), u01(r.z), u01(r.w)};
}

// ---------------------------------------------------------------------------
// small vector algebra
// ---------------------------------------------------------------------------
struct f3 { float x, y, z; };
__device__ __forceinline__ f3 operator+(f3 a, f3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ f3 operator-(f3 a, f3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ f3 operator*(float s, f3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ float dot(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ f3 cross(f3 a, f3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
// Hardware square root and reciprocal (about 1 ulp).  The compiler wraps
// sqrtf and 1/x in range scaling for denormal arguments (five or six
// instructions instead of one); the arguments below are normal numbers or
// zero, where the bare instruction gives the same result.
__device__ __forceinline__ float hw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float hw_div(float a, float b) { return a * hw_rcp(b); }
__device__ __forceinline__ f3 normalize(f3 a) { return hw_rcp(hw_sqrt(dot(a, a))) * a; }
__device__ __forceinline__ bool finite3(f3 a) {
  return isfinite(a.x) && isfinite(a.y) && isfinite(a.z);
}
__device__ __forceinline__ float comp(f3 a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }

// orthonormal basis of a unit vector (Duff et al., JCGT 2017) with the branch
// switched at n_z = -1/2: for normals in the xy plane (detector walls) the sign
// of n_z is rounding noise and must not select the basis
__device__ __forceinline__ void onb(f3 n, f3& b1, f3& b2) {
  const float s = n.z >= -0.5f ? 1.0f : -1.0f;
  const float a = -hw_rcp(s + n.z);
  const float b = n.x * n.y * a;
  b1 = {1.0f + s * n.x * n.x * a, s * b, -s * n.x};
  b2 = {b, s + n.y * n.y * a, -n.y};
}

// sin(2 pi u) and cos(2 pi u) by the hardware instructions, which take their
// argument in revolutions: one instruction each instead of the library's
// range reduction and polynomials, with a maximal absolute error of 2.7e-7
// over the uniforms u01 produces (the library's sincospif: 2.0e-7)
__device__ __forceinline__ void sincos_rev(float u, float& s, float& c) {
  s = __builtin_amdgcn_sinf(u);
  c = __builtin_amdgcn_cosf(u);
}

__device__ __forceinline__ f3 isotropic(float u0, float u1) {
  const float c = 1.0f - 2.0f * u0;
  const float s = hw_sqrt(fmaxf(0.0f, (1.0f - c) * (1.0f + c)));
  float sp, cp;
  sincos_rev(u1, sp, cp);
  return {s * cp, s * sp, c};
}

__device__ __forceinline__ f3 random_polarization(f3 d, float u) {
  f3 b1, b2;
  onb(d, b1, b2);
  float sp, cp;
  sincos_rev(u, sp, cp);
  return cp * b1 + sp * b2;
}

// ---------------------------------------------------------------------------
// photon state
// ---------------------------------------------------------------------------
struct Photon {
  f3 pos, dir, pol;
  float time;
  float wavelength;  // nm
  int32_t medium, last_tri, steps, flag, event, sensor;
  float path_len;   // in the gradient material
  int32_t n_sca;    // Rayleigh scatters in the gradient material
  float sum_inv_r, sum_inv_t;
};

enum : int32_t {
  F_DETECT = 1, F_SENSOR_ABSORB = 2, F_SURFACE_ABSORB = 3, F_BULK_ABSORB = 4, F_ESCAPED = 5,
  F_MAX_STEPS = 6, F_NAN_ABORT = 7, F_GEOM = 0x100
};

// dipole Rayleigh scattering: isotropic trial k', keep with probability
// 1 - (e.k')^2; new polarization = e projected off k' (trial 64 kept if all
// fail).  Trial j uses Philox block (step, 2 + j); r is trial 0's block.
__device__ __forceinline__ void rayleigh(Photon& p, uint32_t s0, uint32_t s1, uint64_t pid,
                                         uint32_t step, R4 r) {
  f3 k, e;
  for (uint32_t j = 0;;) {
    k = isotropic(r.u0, r.u1);
    const float ek = dot(p.pol, k);
    e = p.pol - ek * k;
    if (r.u2 < 1.0f - ek * ek || ++j == 64u) break;
    r = draw(s0, s1, pid, step, 2u + j);
  }
  p.dir = k;
  p.pol = normalize(e);
}

// Lambertian reflection into the hemisphere of n_out, fresh polarization
__device__ __forceinline__ void lambertian(Photon& p, f3 n_out, const R4& r) {
  f3 b1, b2;
  onb(n_out, b1, b2);
  const float ct = hw_sqrt(r.u0);
  const float st = hw_sqrt(fmaxf(0.0f, 1.0f - r.u0));
  float sp, cp;
  sincos_rev(r.u1, sp, cp);
  p.dir = normalize((st * cp) * b1 + (st * sp) * b2 + ct * n_out);
  p.pol = random_polarization(p.dir, r.u2);
}

// mirror reflection about the plane of unit normal n (defined at normal incidence)
__device__ __forceinline__ void specular(Photon& p, f3 n) {
  p.dir = normalize(p.dir - (2.0f * dot(p.dir, n)) * n);
  p.pol = normalize(p.pol - (2.0f * dot(p.pol, n)) * n);
}

// Fresnel at a real-index boundary; nhat points back into the incident medium.
// Returns true if transmitted.
__device__ __forceinline__ bool fresnel(Photon& p, f3 nhat, float n1, float n2, float u) {
  const f3 d = p.dir, e = p.pol;
  const float ci = -dot(d, nhat);
  const float eta = hw_div(n1, n2);
  const float st2 = eta * eta * (1.0f - ci * ci);
  if (st2 >= 1.0f) {
    specular(p, nhat);
    return false;
  }
  // 1 - st2 >= 2^-24 here, and the denominators are positive
  const float ct = hw_sqrt(1.0f - st2);
  const float rs = hw_div(n1 * ci - n2 * ct, n1 * ci + n2 * ct);
  const float rp = hw_div(n2 * ci - n1 * ct, n2 * ci + n1 * ct);
  const float ts = hw_div(2.0f * n1 * ci, n1 * ci + n2 * ct);
  const float tp = hw_div(2.0f * n1 * ci, n2 * ci + n1 * ct);
  const f3 sv = cross(d, nhat);
  const float sl = hw_sqrt(dot(sv, sv));
  const f3 s = (sl < 1e-6f) ? e : hw_rcp(sl) * sv;
  const float as = dot(e, s);
  const float ap = dot(e, cross(s, d));
  const float R = as * as * rs * rs + ap * ap * rp * rp;
  if (u < R) {
    const f3 dr = normalize(d + (2.0f * ci) * nhat);
    p.pol = normalize((rs * as) * s + (rp * ap) * cross(s, dr));
    p.dir = dr;
    return false;
  }
  const f3 dt = normalize(eta * d + (eta * ci - ct) * nhat);
  p.pol = normalize((ts * as) * s + (tp * ap) * cross(s, dt));
  p.dir = dt;
  return true;
}

// ---------------------------------------------------------------------------
// wavelength dependence: dispersion tables, complex-index and thin-film surfaces
// ---------------------------------------------------------------------------

// Material at wavelength lam: the index and the attenuation coefficients 1/L
// interpolated linearly between the neighbouring samples of its table, held
// constant outside (materials without a table: their table entry).
__device__ __forceinline__ DevMaterial material_at(const LaunchArgs& a, int32_t m, float lam) {
  DevMaterial r = a.mats[m];
  if (a.dispersive != 0 && ((a.dispersive >> m) & 1)) {
    const DevDispersion& t = a.disp[m];
    float n, ia, ir;
    if (lam <= t.lambda[0]) {
      n = t.index[0]; ia = t.inv_abs[0]; ir = t.inv_ray[0];
    } else if (lam >= t.lambda[t.n - 1]) {
      n = t.index[t.n - 1]; ia = t.inv_abs[t.n - 1]; ir = t.inv_ray[t.n - 1];
    } else {
      int32_t i = 0;
      while (t.lambda[i + 1] < lam) ++i;
      const float w = hw_div(lam - t.lambda[i], t.lambda[i + 1] - t.lambda[i]);
      n = t.index[i] + w * (t.index[i + 1] - t.index[i]);
      ia = t.inv_abs[i] + w * (t.inv_abs[i + 1] - t.inv_abs[i]);
      ir = t.inv_ray[i] + w * (t.inv_ray[i + 1] - t.inv_ray[i]);
    }
    r.n = n;
    r.abs_len = ia > 0.0f ? hw_rcp(ia) : kInfF;
    r.ray_len = ir > 0.0f ? hw_rcp(ir) : kInfF;
  }
  return r;
}

// minimal complex arithmetic in FP32
struct cf { float re, im; };
__device__ __forceinline__ cf c_add(cf a, cf b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cf c_sub(cf a, cf b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cf c_mul(cf a, cf b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cf c_div(cf a, cf b) {
  const float d = 1.0f / (b.re * b.re + b.im * b.im);
  return {(a.re * b.re + a.im * b.im) * d, (a.im * b.re - a.re * b.im) * d};
}
// principal square root (Re >= 0, the sign of Im follows the argument's)
__device__ __forceinline__ cf c_sqrt(cf z) {
  const float r = hypotf(z.re, z.im);
  if (r == 0.0f) return {0.0f, 0.0f};
  if (z.re >= 0.0f) {
    const float t = sqrtf(0.5f * (r + z.re));
    return {t, z.im / (2.0f * t)};
  }
  const float t = sqrtf(0.5f * (r - z.re));
  return {fabsf(z.im) / (2.0f * t), copysignf(t, z.im)};
}
__device__ __forceinline__ float c_norm(cf z) { return z.re * z.re + z.im * z.im; }

// Amplitude reflection coefficients (s, p) from a medium of index n1 at
// incidence cosine ci on a medium of complex index (model COMPLEX_INDEX) or on
// a film over it (THIN_FILM, phase 2 pi d q_f / lam): with
// q_j = sqrt(n_j^2 - n1^2 sin^2), r_s = (q_a - q_b) / (q_a + q_b) and
// r_p = (n_b^2 q_a - n_a^2 q_b) / (n_b^2 q_a + n_a^2 q_b) per interface, and
// r = (r_01 + r_12 E) / (1 + r_01 r_12 E), E = exp(2 i phase), for the film.
__device__ __forceinline__ void film_reflection(int32_t model, float n1, float ci, float n_re,
                                                float n_im, float nf, float two_pi_d, float lam,
                                                cf& rs, cf& rp) {
  const float s2 = n1 * n1 * (1.0f - ci * ci);
  const cf q1{n1 * ci, 0.0f};
  const cf e1{n1 * n1, 0.0f};
  const cf e2{n_re * n_re - n_im * n_im, 2.0f * n_re * n_im};
  const cf q2 = c_sqrt(cf{e2.re - s2, e2.im});
  if (model == XP_SURF_COMPLEX_INDEX) {
    rs = c_div(c_sub(q1, q2), c_add(q1, q2));
    rp = c_div(c_sub(c_mul(e2, q1), c_mul(e1, q2)), c_add(c_mul(e2, q1), c_mul(e1, q2)));
    return;
  }
  const cf ef{nf * nf, 0.0f};
  const cf qf = c_sqrt(cf{ef.re - s2, 0.0f});
  const cf r01s = c_div(c_sub(q1, qf), c_add(q1, qf));
  const cf r12s = c_div(c_sub(qf, q2), c_add(qf, q2));
  const cf r01p = c_div(c_sub(c_mul(ef, q1), c_mul(e1, qf)), c_add(c_mul(ef, q1), c_mul(e1, qf)));
  const cf r12p = c_div(c_sub(c_mul(e2, qf), c_mul(ef, q2)), c_add(c_mul(e2, qf), c_mul(ef, q2)));
  // E = exp(2 i k qf), k = 2 pi d / lam: modulus exp(-2 k Im qf), phase 2 k Re qf
  const float k = two_pi_d / lam;
  const float mag = expf(-2.0f * k * qf.im);
  float sp, cp;
  sincosf(2.0f * k * qf.re, &sp, &cp);
  const cf E{mag * cp, mag * sp};
  const cf one{1.0f, 0.0f};
  rs = c_div(c_add(r01s, c_mul(r12s, E)), c_add(one, c_mul(c_mul(r01s, r12s), E)));
  rp = c_div(c_add(r01p, c_mul(r12p, E)), c_add(one, c_mul(c_mul(r01p, r12p), E)));
}

// Reflection off a complex-index / thin-film surface with probability
// a_s^2 |r_s|^2 + a_p^2 |r_p|^2; the reflected photon keeps a linear
// polarization, its s and p parts scaled by |r| with the sign of Re r.
// Returns true if reflected.
__device__ __forceinline__ bool model_reflection(Photon& p, f3 nhat, float n1, const DevSurface& s,
                                                 float u) {
  const f3 d = p.dir, e = p.pol;
  const float ci = -dot(d, nhat);
  cf rs, rp;
  film_reflection(s.model, n1, ci, s.n_re, s.n_im, s.film_n, s.two_pi_d, p.wavelength, rs, rp);
  const f3 sv = cross(d, nhat);
  const float sl = sqrtf(dot(sv, sv));
  const f3 sd = (sl < 1e-6f) ? e : (1.0f / sl) * sv;
  const float as = dot(e, sd);
  const float ap = dot(e, cross(sd, d));
  const float R = as * as * c_norm(rs) + ap * ap * c_norm(rp);
  if (!(u < R)) return false;
  const f3 dr = normalize(d + (2.0f * ci) * nhat);
  const float ms = copysignf(sqrtf(c_norm(rs)), rs.re);
  const float mp = copysignf(sqrtf(c_norm(rp)), rp.re);
  p.pol = normalize((ms * as) * sd + (mp * ap) * cross(sd, dr));
  p.dir = dr;
  return true;
}

// ---------------------------------------------------------------------------
// ray / triangle (watertight, Woop, Benthin and Wald, JCGT 2013), FP32
// ---------------------------------------------------------------------------
// The ray in the frame of its dominant axis kz: origin rotated to
// (kx, ky, kz) = (kz + 1, kz + 2, kz) mod 3, shear constants, and the first
// record of the triangle copy rotated the same way.  The method swaps kx and ky
// when d_kz < 0 to keep the winding; without the swap u, v, w, the determinant
// and the distance numerator are all exactly negated (the products are not
// contracted), which changes neither the inside test nor the distance.
struct RayW {
  f3 o;           // rotated origin
  float sx, sy, sz;
  uint32_t toff;  // byte offset of the rotated triangle copy (records are 48 bytes)
};

__device__ __forceinline__ RayW make_ray(f3 o, f3 d, int32_t n_tris) {
  RayW r;
  const float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
  const int kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
  const int kx = kz == 2 ? 0 : kz + 1;
  const int ky = kx == 2 ? 0 : kx + 1;
  r.o = f3{comp(o, kx), comp(o, ky), comp(o, kz)};
  const float dz = comp(d, kz);
  r.sx = hw_div(comp(d, kx), dz);
  r.sy = hw_div(comp(d, ky), dz);
  r.sz = hw_rcp(dz);
  r.toff = uint32_t(kx) * uint32_t(n_tris) * 48u;  // (kz + 1) mod 3 == kx
  return r;
}

// hit distance or +inf; products are never contracted so that the edge
// function of a shared edge is exactly negated between its two triangles
__device__ __forceinline__ float intersect(const RayW& r, const float* va, const float* vb,
                                           const float* vc) {
  // vertices already rotated to (kx, ky, kz)
  const f3 a{va[0] - r.o.x, va[1] - r.o.y, va[2] - r.o.z};
  const f3 b{vb[0] - r.o.x, vb[1] - r.o.y, vb[2] - r.o.z};
  const f3 c{vc[0] - r.o.x, vc[1] - r.o.y, vc[2] - r.o.z};
  const float akz = a.z, bkz = b.z, ckz = c.z;
  const float ax = fmaf(-r.sx, akz, a.x), ay = fmaf(-r.sy, akz, a.y);
  const float bx = fmaf(-r.sx, bkz, b.x), by = fmaf(-r.sy, bkz, b.y);
  const float cx = fmaf(-r.sx, ckz, c.x), cy = fmaf(-r.sy, ckz, c.y);
  const float u = __fsub_rn(__fmul_rn(cx, by), __fmul_rn(cy, bx));
  const float v = __fsub_rn(__fmul_rn(ax, cy), __fmul_rn(ay, cx));
  const float w = __fsub_rn(__fmul_rn(bx, ay), __fmul_rn(by, ax));
  // mixed edge signs: outside.  Written without branches: the wave runs the
  // test for every lane anyway, and the exec-mask branches cost more than the
  // distance computed for lanes that then discard it.
  const bool neg = (u < 0.0f) | (v < 0.0f) | (w < 0.0f);
  const bool pos = (u > 0.0f) | (v > 0.0f) | (w > 0.0f);
  const float det = __fadd_rn(__fadd_rn(u, v), w);
  const float az = r.sz * akz, bz = r.sz * bkz, cz = r.sz * ckz;
  const float t = __fadd_rn(__fadd_rn(__fmul_rn(u, az), __fmul_rn(v, bz)), __fmul_rn(w, cz));
  const bool inside = !(neg & pos) & (det != 0.0f);
  return inside ? t * __builtin_amdgcn_rcpf(det) : kInfF;  // hardware reciprocal, 1 ulp
}

struct Best {
  float t;
  int32_t tri;   // mesh triangle index (-1: none)
  int32_t rec;   // record index
};

// Records are addressed by 32-bit byte offsets from the array start (fewer
// than 2^24 references per copy, so record index x 48 fits a 24-bit multiply
// and the three copies fit 4 GB).
__device__ __forceinline__ void test_triangle(const TriRec* __restrict__ tris, int32_t k,
                                              const RayW& r, float tmin, int32_t skip, Best& b) {
  const char* base = reinterpret_cast<const char*>(tris);
  const uint32_t off = __umul24(uint32_t(k), 48u) + r.toff;  // the copy rotated for this ray
  const float4 A = *reinterpret_cast<const float4*>(base + off);
  const float4 B = *reinterpret_cast<const float4*>(base + off + 16u);
  const float4 C = *reinterpret_cast<const float4*>(base + off + 32u);
  const int32_t id = __float_as_int(A.w);
  const float va[3] = {A.x, A.y, A.z}, vb[3] = {B.x, B.y, B.z}, vc[3] = {C.x, C.y, C.z};
  const float t = intersect(r, va, vb, vc);
  // The closest hit orders by (distance, triangle index): for distances >= 0
  // the float bits order as the values do, so the pair is one 64-bit key, and
  // "nearer, or as near with a lower index" is one unsigned comparison.  No
  // hit yet has index -1 (all ones), so any hit at the search bound itself
  // is taken.  The skipped triangle is rejected only here (an early return on
  // its id lets the compiler load the id alone first, a second memory round
  // trip); selects instead of branches.
  const uint64_t key = (uint64_t(__float_as_uint(t)) << 32) | uint32_t(id);
  const uint64_t best = (uint64_t(__float_as_uint(b.t)) << 32) | uint32_t(b.tri);
  const bool take = (id != skip) & (t > tmin) & (t < kInfF) & (key < best);
  b.t = take ? t : b.t;
  b.tri = take ? id : b.tri;
  b.rec = take ? k : b.rec;
}

struct Counters {
  uint32_t nodes, tris;
  uint32_t slots, busy;  // search lane slots offered / used (SIMD utilization)
};

// Node fetch: the first n_lds nodes (the top levels, breadth-first) are read
// from LDS, where they start at byte address lds_base (a multiple of 128:
// 0, or the size of the block tallies before them), the rest from global
// memory.  The box planes are fetched in the order the ray meets them (near
// before far on each axis, by the signs of its direction), so the slab test
// needs no per-axis min / max: with a non-negative reciprocal the lower
// plane's entry distance is the smaller one (rounding is monotone), and the
// reciprocals are never zero.  Both paths read the node at the same byte
// offsets, the global path from a base moved back by lds_base: a node is
// 128 bytes, each axis's lower and upper planes 16 bytes apart in a 32-byte
// pair, so the near plane is at (node << 7) + lds_base | 16 * sign and the
// far plane at that offset ^ 16.
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) const f4v lds_f4;
__device__ __forceinline__ void fetch_node(const Node4* __restrict__ gnodes, int32_t n_lds,
                                           uint32_t lds_base, int32_t node, f3 inv,
                                           float4 (&q)[7]) {
  const uint32_t base = (uint32_t(node) << 7) + lds_base;
  const uint32_t xn = base | ((__float_as_uint(inv.x) >> 31) << 4);
  const uint32_t yn = base | ((__float_as_uint(inv.y) >> 31) << 4);
  const uint32_t zn = base | ((__float_as_uint(inv.z) >> 31) << 4);
  // q[0..5] = near x, far x, near y, far y, near z, far z; q[6] = children
  const uint32_t off[7] = {xn, xn ^ 16u, yn + 32u, (yn ^ 16u) + 32u, zn + 64u, (zn ^ 16u) + 64u,
                           base + 96u};
  if (node < n_lds) {
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      const f4v v = *(lds_f4*)(uintptr_t)off[i];
      q[i] = make_float4(v.x, v.y, v.z, v.w);
    }
  } else {
    const char* g = reinterpret_cast<const char*>(gnodes) - lds_base;
#pragma unroll
    for (int i = 0; i < 7; ++i) q[i] = *reinterpret_cast<const float4*>(g + off[i]);
  }
}

typedef __attribute__((address_space(3))) int32_t lds_i32;

// Per-lane traversal stack: the newest entries in a window of LDS slots (slot
// k of a lane at bottom + 64 k, the 64 lanes of a wave side by side), the
// older ones in this lane's column of a global overflow array.  A node visit
// first makes room for its (at most four) pushes: if the window holds more
// than `limit` entries, all of them move to the overflow array (rare: the
// stack is seldom deeper than a few entries); pops read the overflow array
// while the window is empty.  Pushes and pops move one LDS address.  `total`
// is the host-computed worst case; a visit that would exceed it fails.
struct LaneStack {
  lds_i32* bottom;     // this lane's window slot 0
  lds_i32* top;        // the first free window slot
  int32_t limit;       // 256 * (window slots - 4): bytes of entries that leave four slots free
  int32_t* glob;       // this lane's overflow column: entry k at glob[k * gstride]
  int64_t gstride;
  int32_t total;
  int32_t sp;          // entries in use, window and overflow
  __device__ __forceinline__ void clear() {
    sp = 0;
    top = bottom;
  }
  // make room for four entries in the window
  __device__ __forceinline__ void reserve4() {
    // bytes between the 32-bit LDS addresses: 256 per entry
    const int32_t held = int32_t((uint32_t)(uintptr_t)top - (uint32_t)(uintptr_t)bottom);
    if (held > limit) {
      const int32_t first = sp - (held >> 8);  // stack index of window slot 0
      for (int32_t k = 0; k < (held >> 8); ++k) glob[int64_t(first + k) * gstride] = bottom[64 * k];
      top = bottom;
    }
  }
  // write entry j (< 4) above the top; valid after reserve4
  __device__ __forceinline__ void put(int32_t j, int32_t e) { top[j * 64] = e; }
  // the n entries written above the top join the stack
  __device__ __forceinline__ void advance(int32_t n) {
    top += n * 64;
    sp += n;
  }
  __device__ __forceinline__ int32_t pop() {
    --sp;
    if (top == bottom) return glob[int64_t(sp) * gstride];
    top -= 64;
    return *top;
  }
};

// Visit one inner node: test its four child boxes, follow the nearest hit if
// it is an inner node or hold it if it is a leaf, and push the other hits.
// Stack entries are node indices (>= 0) or complemented packed leaves
// (first << 3 | count - 1).  Returns false if the stack bound is exceeded.
template <bool kCount>
__device__ __forceinline__ bool visit_node(const Node4* __restrict__ gnodes, int32_t n_lds,
                                           uint32_t lds_base, f3 inv, f3 oi,
                                           float tmax, LaneStack& st, int32_t& node,
                                           int32_t& leaf, Counters& cnt) {
  float4 q[7];
  fetch_node(gnodes, n_lds, lds_base, node, inv, q);
  __builtin_amdgcn_s_setprio(1);  // the node's loads are issued
  if (kCount) cnt.nodes++;
  const float lox[4] = {q[0].x, q[0].y, q[0].z, q[0].w};  // near planes
  const float hix[4] = {q[1].x, q[1].y, q[1].z, q[1].w};  // far planes
  const float loy[4] = {q[2].x, q[2].y, q[2].z, q[2].w};
  const float hiy[4] = {q[3].x, q[3].y, q[3].z, q[3].w};
  const float loz[4] = {q[4].x, q[4].y, q[4].z, q[4].w};
  const float hiz[4] = {q[5].x, q[5].y, q[5].z, q[5].w};
  const int32_t child[4] = {__float_as_int(q[6].x), __float_as_int(q[6].y),
                            __float_as_int(q[6].z), __float_as_int(q[6].w)};
  // Each hit child's entry distance (>= 0, so its bits order as the value
  // does) with the child's slot in the two low bits; a miss is all ones.  The
  // smallest key is the nearest hit (ties, and distances within 4 ulp, go to
  // the lower slot), found with two integer minima instead of sorting.
  uint32_t key[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float t0x = fmaf(lox[i], inv.x, -oi.x), t1x = fmaf(hix[i], inv.x, -oi.x);
    const float t0y = fmaf(loy[i], inv.y, -oi.y), t1y = fmaf(hiy[i], inv.y, -oi.y);
    const float t0z = fmaf(loz[i], inv.z, -oi.z), t1z = fmaf(hiz[i], inv.z, -oi.z);
    const float tn = fmaxf(fmaxf(t0x, t0y), fmaxf(t0z, 0.0f));
    const float tf = fminf(fminf(t1x, t1y), fminf(t1z, tmax));
    // empty slots hold an inverted box (lo = +inf, hi = -inf), which every
    // slab test misses: no separate check of the child entry
    const bool hit = tn <= tf * 1.0000005f;
    key[i] = hit ? ((__float_as_uint(tn) & ~3u) | uint32_t(i)) : ~0u;
  }
  const uint32_t nearest = min(min(key[0], key[1]), min(key[2], key[3]));
  const uint32_t j = nearest & 3u;
  // every other hit is pushed (the lower slots on top); the nearest is
  // followed if it is an inner node and held if it is a leaf.  Writes go to
  // the slot above the top whether or not they count, so no branches.
  st.reserve4();
  int32_t npush = 0;
  int32_t near_entry = child[3];
#pragma unroll
  for (int i = 3; i >= 0; --i) {
    const bool is_nearest = j == uint32_t(i);
    near_entry = is_nearest ? child[i] : near_entry;
    st.put(npush, child[i]);
    npush += ((key[i] != ~0u) & !is_nearest) ? 1 : 0;
  }
  const bool any = nearest != ~0u;
  const bool near_leaf = any & (near_entry < 0);
  // a nearest leaf while the lane still holds one (leaves of several
  // triangles): the held leaf goes to the stack
  if (near_leaf & (leaf >= 0)) {
    st.put(npush, ~leaf);
    ++npush;
  }
  node = (any & (near_entry >= 0)) ? near_entry : -1;
  leaf = near_leaf ? ~near_entry : leaf;
  if (st.sp + npush > st.total) return false;
  st.advance(npush);
  return true;
}

// BVH closest hit: t in (tmin, b.t], ties to the lower triangle index, for
// the closest-hit test hook (the transport kernel runs the same node visits
// and triangle tests as micro-steps of its lane state machine).
//
// Two phases that the lanes of a wave run in step.  Node phase: each lane
// without a postponed leaf visits inner nodes (popping its stack when it has
// none) until every lane of the wave holds a leaf or has run out of work.
// Leaf phase: every lane holding a leaf tests its triangles.  Running the
// phases separately keeps the wave's lanes on the same code (node tests or
// triangle tests) instead of paying for both in every iteration.
// Returns false only if the stack would overflow its host-computed bound.
template <bool kCount>
__device__ __forceinline__ bool traverse(const Node4* __restrict__ gnodes, int32_t n_lds,
                                         const TriRec* __restrict__ tris,
                                         int32_t n_tris, LaneStack st, f3 o, f3 d, float tmin,
                                         int32_t skip, Best& b, Counters& cnt) {
  const RayW ray = make_ray(o, d, n_tris);
  const float tiny = 1e-30f;
  const f3 inv{hw_rcp(fabsf(d.x) > tiny ? d.x : copysignf(tiny, d.x)),
               hw_rcp(fabsf(d.y) > tiny ? d.y : copysignf(tiny, d.y)),
               hw_rcp(fabsf(d.z) > tiny ? d.z : copysignf(tiny, d.z))};
  const f3 oi{o.x * inv.x, o.y * inv.y, o.z * inv.z};
  int32_t node = 0;   // inner node to visit next, or -1
  int32_t leaf = -1;  // postponed leaf (packed), or -1
  bool ok = true;
  st.clear();
  while (true) {
    // ---- node phase ----
    while (true) {
      const bool active = leaf < 0 && (node >= 0 || st.sp > 0);
      if (kCount) {
        cnt.slots++;
        if (active) cnt.busy++;
      }
      if (active) {
        if (node < 0) {
          const int32_t e = st.pop();
          if (e >= 0) node = e; else leaf = ~e;
        }
        if (node >= 0 && leaf < 0) {
          if (!visit_node<kCount>(gnodes, n_lds, 0u, inv, oi, b.t, st, node, leaf, cnt)) {
            ok = false;
            node = -1;
            leaf = -1;
            st.clear();
          }
        }
      }
      if (__ballot(leaf < 0 && (node >= 0 || st.sp > 0)) == 0ull) break;
    }
    // ---- leaf phase ----
    if (leaf >= 0) {
      const int32_t first = leaf >> 3, n = (leaf & 7) + 1;
      for (int32_t k = first; k < first + n; ++k) {
        if (kCount) cnt.tris++;
        test_triangle(tris, k, ray, tmin, skip, b);
      }
      leaf = -1;
    }
    if (__ballot(node >= 0 || st.sp > 0) == 0ull) break;
  }
  return ok;
}

// ---------------------------------------------------------------------------
// sources
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t source_of(const LaunchArgs& a, int64_t i) {
  if (a.offsets == nullptr) return i / a.count_per_source;
  int64_t lo = 0, hi = a.n_sources;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (a.offsets[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int64_t uniform64(int64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(x)));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(x) >> 32));
  return int64_t((uint64_t(hi) << 32) | lo);
}

// Source of photon i for sources with prefix offsets (the last source s with
// offsets[s] <= i), with i the same in every lane of the wave: a 64-ary
// search in which every lane loads one offset of the bracket per round and a
// ballot finds the last one not past i (offsets increase, so the lanes that
// find offsets[s] <= i are a prefix of the wave), two dependent loads for up
// to 4,096 sources instead of twelve in a binary search.
__device__ __forceinline__ int64_t wave_source_of(const LaunchArgs& a, int64_t i, uint32_t lane) {
  i = uniform64(i);
  int64_t lo = 0, n = uniform64(a.n_sources);  // the source lies in [lo, lo + n)
  while (n > 1) {
    const int64_t step = (n + 63) >> 6;  // sources per lane
    const int64_t s = lo + int64_t(lane) * step;
    const bool le = s < lo + n && a.offsets[s] <= i;
    const uint64_t m = __ballot(le);       // bit 0 is set: offsets[lo] <= i
    const int64_t k = 63 - __clzll(m);     // the last lane with offsets[s] <= i
    const int64_t nlo = lo + k * step;
    n = min(step, lo + n - nlo);
    lo = nlo;
  }
  return lo;
}

// Emission time from the two-component scintillation decay: Philox block
// (step 0, sub 2), u0 picks the singlet state with its fraction, u1 the decay.
__device__ __forceinline__ float emission_time(uint32_t s0, uint32_t s1, uint64_t pid,
                                               float tau_singlet, float tau_triplet,
                                               float singlet_fraction, bool& singlet) {
  const R4 r = draw(s0, s1, pid, 0u, 2u);
  singlet = r.u0 < singlet_fraction;
  return -(singlet ? tau_singlet : tau_triplet) * logf(r.u1);
}

// Wavelength from the Gaussian emission spectrum: Philox block (step 0,
// sub 3), Box-Muller.
__device__ __forceinline__ float emission_wavelength(uint32_t s0, uint32_t s1, uint64_t pid,
                                                     float mean, float sigma) {
  if (!(sigma > 0.0f)) return mean;
  const R4 r = draw(s0, s1, pid, 0u, 3u);
  return mean + sigma * sqrtf(-2.0f * logf(r.u0)) * cospif(2.0f * r.u1);
}

// Uniform point of the cylinder r <= cyl_r, zlo <= z <= zhi: Philox block
// (step 0, sub 1), r = cyl_r sqrt(u0), phi = 2 pi u1, z = zlo + (zhi - zlo) u2.
__device__ __forceinline__ f3 cylinder_point(uint32_t s0, uint32_t s1, uint64_t pid, float cyl_r,
                                             float zlo, float zhi) {
  const R4 q = draw(s0, s1, pid, 0u, 1u);
  const float rr = cyl_r * hw_sqrt(q.u0);
  float sp, cp;
  sincos_rev(q.u1, sp, cp);
  return {rr * cp, rr * sp, zlo + (zhi - zlo) * q.u2};
}

// Emit photon i (launch-local) with id pid; src, when >= 0, is its source
// (POINTS), already known to the caller.
__device__ __forceinline__ void emit(Photon& p, const LaunchArgs& a, int64_t i, uint64_t pid,
                                     int64_t src = -1) {
  p.time = 0.0f;
  p.wavelength = emission_wavelength(a.seed_lo, a.seed_hi, pid, a.wl_mean, a.wl_sigma);
  if (a.time_profile == XP_TIME_SCINTILLATION) {
    bool singlet;
    p.time = emission_time(a.seed_lo, a.seed_hi, pid, a.tau_singlet, a.tau_triplet,
                           a.singlet_fraction, singlet);
  }
  p.medium = a.medium;
  p.last_tri = -1;
  p.steps = 0;
  p.flag = 0;
  p.event = 0;
  p.sensor = -1;
  p.path_len = 0.0f;
  p.n_sca = 0;
  p.sum_inv_r = 0.0f;
  p.sum_inv_t = 0.0f;
  if (a.src_kind == XP_SRC_EXPLICIT) {
    p.pos = {a.positions[3 * i], a.positions[3 * i + 1], a.positions[3 * i + 2]};
    p.dir = normalize(f3{a.dirs[3 * i], a.dirs[3 * i + 1], a.dirs[3 * i + 2]});
    const f3 e{a.pols[3 * i], a.pols[3 * i + 1], a.pols[3 * i + 2]};
    p.pol = normalize(e - dot(e, p.dir) * p.dir);
    return;
  }
  const R4 r = draw(a.seed_lo, a.seed_hi, pid, 0u, 0u);
  p.dir = isotropic(r.u0, r.u1);
  p.pol = random_polarization(p.dir, r.u2);
  if (a.src_kind == XP_SRC_POINTS) {
    const int64_t s = src >= 0 ? src : source_of(a, i);
    p.pos = {a.positions[3 * s], a.positions[3 * s + 1], a.positions[3 * s + 2]};
    p.event = a.per_source_events ? int32_t(s) : 0;
  } else {
    p.pos = cylinder_point(a.seed_lo, a.seed_hi, pid, a.cyl_r, a.cyl_zlo, a.cyl_zhi);
  }
}

// ---------------------------------------------------------------------------
// one transport step, in two halves around the closest-hit search
// ---------------------------------------------------------------------------
struct StepDraw {
  float d_abs, d_sca, u2;  // free paths to absorption and scattering; decision uniform
};

// Start step s = steps + 1: draw the free paths in the current medium.
__device__ __forceinline__ StepDraw begin_step(Photon& p, const LaunchArgs& a, uint64_t pid) {
  const int32_t step = ++p.steps;
  const DevMaterial m = material_at(a, p.medium, p.wavelength);
  const R4 r = draw(a.seed_lo, a.seed_hi, pid, uint32_t(step), 0u);
  StepDraw sd;
  sd.d_abs = isinf(m.abs_len) ? kInfF : -m.abs_len * logf(r.u0);
  sd.d_sca = isinf(m.ray_len) ? kInfF : -m.ray_len * logf(r.u1);
  sd.u2 = r.u2;
  return sd;
}

// Finish the step given the closest hit b within min(d_abs, d_sca) (b.tri < 0:
// none; b.tri == kTraversalFailed: the stack bound was exceeded).  Returns
// true when the photon has ended.
constexpr int32_t kTraversalFailed = -2;

template <bool kGradAcc>
__device__ __forceinline__ bool finish_step(Photon& p, const LaunchArgs& a, uint64_t pid,
                                            const StepDraw& sd, const Best& b) {
  if (b.tri == kTraversalFailed) {
    p.flag |= F_NAN_ABORT;  // prevented by the host's stack sizing
    return true;
  }
  const int32_t step = p.steps;
  const DevMaterial m = material_at(a, p.medium, p.wavelength);
  // the interaction's first random block, drawn for every lane at once: the
  // Lambertian block (sub 1) of a surface event, Rayleigh trial 0 (sub 2) of
  // a bulk event (one Philox pass instead of one per kind of interaction)
  const R4 r1 = draw(a.seed_lo, a.seed_hi, pid, uint32_t(step), b.tri < 0 ? 2u : 1u);
  const float d_abs = sd.d_abs, d_sca = sd.d_sca;
  const float d_bulk = fminf(d_abs, d_sca);
  const bool in_grad = p.medium == a.grad_material;
  if (b.tri < 0) {
    if (isinf(d_bulk)) {
      p.flag |= F_ESCAPED;
      return true;
    }
    p.pos = p.pos + d_bulk * p.dir;
    p.time += hw_div(d_bulk * m.n, kCns);
    if (kGradAcc && in_grad) p.path_len += d_bulk;
    if (d_abs <= d_sca) {
      p.flag |= F_BULK_ABSORB;
      return true;
    }
    if (kGradAcc && in_grad) p.n_sca += 1;
    rayleigh(p, a.seed_lo, a.seed_hi, pid, uint32_t(step), r1);
    p.last_tri = -1;
  } else {
    const int32_t k = b.tri;
    p.pos = p.pos + b.t * p.dir;
    p.time += hw_div(b.t * m.n, kCns);
    if (kGradAcc && in_grad) p.path_len += b.t;
    const float4 A = *reinterpret_cast<const float4*>(a.tris[b.rec].a);
    const float4 B = *reinterpret_cast<const float4*>(a.tris[b.rec].b);
    const float4 C = *reinterpret_cast<const float4*>(a.tris[b.rec].c);
    const f3 v0{A.x, A.y, A.z};
    const f3 N = normalize(cross(f3{B.x, B.y, B.z} - v0, f3{C.x, C.y, C.z} - v0));
    const uint32_t packed = __float_as_uint(B.w);
    const int32_t sensor = __float_as_int(C.w);
    const int32_t mat_in = int32_t(packed & 0xffu), mat_out = int32_t((packed >> 8) & 0xffu);
    const int32_t si = int32_t(packed >> 16) - 1;
    const bool from_outer = dot(p.dir, N) < 0.0f;
    const int32_t m_from = from_outer ? mat_out : mat_in;
    const int32_t m_to = from_outer ? mat_in : mat_out;
    if (m_from != p.medium) {
      p.flag |= F_GEOM;
      p.medium = m_from;
    }
    const f3 n_back = from_outer ? N : (-1.0f) * N;
    p.last_tri = k;
    if (si >= 0) {
      const DevSurface s = a.surfs[si];
      const int32_t sflags = s.flags_grad & 0xff;
      const int32_t gpar = (s.flags_grad >> 8) - 1;
      const bool is_sensor = sensor >= 0;
      if ((sflags & XP_SURF_DETECT_FRONT_ONLY) && !from_outer) {
        p.flag |= F_SURFACE_ABSORB;
        return true;
      }
      const float u = sd.u2;
      if (s.model != XP_SURF_EXPLICIT) {
        // reflectance from the complex index or the film; a photon that is not
        // reflected enters the surface's material: detected on a sensor
        if (!model_reflection(p, n_back, material_at(a, m_from, p.wavelength).n, s, u)) {
          if (is_sensor) {
            p.flag |= F_DETECT;
            p.sensor = sensor;
          } else {
            p.flag |= F_SURFACE_ABSORB;
          }
          return true;
        }
        p.pos = p.pos + a.surface_offset * n_back;
      } else if (u < s.c_detect) {
        if (is_sensor) {
          p.flag |= F_DETECT;
          p.sensor = sensor;
        } else {
          p.flag |= F_SURFACE_ABSORB;
        }
        return true;
      } else if (u < s.c_absorb) {
        if (is_sensor) {
          p.flag |= F_SENSOR_ABSORB;
          p.sensor = sensor;
        } else {
          p.flag |= F_SURFACE_ABSORB;
        }
        return true;
      } else {
        bool through = false;
        if (u < s.c_diffuse) {
          lambertian(p, n_back, r1);
          if (kGradAcc && gpar == 2) p.sum_inv_r += s.inv_r;
        } else if (u < s.c_specular) {
          specular(p, N);
          if (kGradAcc && gpar == 2) p.sum_inv_r += s.inv_r;
        } else if (s.p_transmit > 0.0f) {
          p.medium = m_to;
          through = true;
          if (kGradAcc && gpar == 3) p.sum_inv_t += s.inv_t;
        } else {
          p.flag |= is_sensor ? F_SENSOR_ABSORB : F_SURFACE_ABSORB;
          if (is_sensor) p.sensor = sensor;
          return true;
        }
        p.pos = p.pos + (through ? -a.surface_offset : a.surface_offset) * n_back;
      }
    } else {
      const float n1 = material_at(a, m_from, p.wavelength).n;
      const float n2 = material_at(a, m_to, p.wavelength).n;
      bool through = true;
      if (n1 != n2) through = fresnel(p, n_back, n1, n2, sd.u2);
      if (through) p.medium = m_to;
      p.pos = p.pos + (through ? -a.surface_offset : a.surface_offset) * n_back;
    }
  }
  if (!finite3(p.pos) || !finite3(p.dir) || !finite3(p.pol)) {
    p.flag |= F_NAN_ABORT;
    return true;
  }
  if (step >= a.max_steps) {
    p.flag |= F_MAX_STEPS;
    return true;
  }
  return false;
}

__device__ __forceinline__ uint32_t lane_rank(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(uint32_t(mask >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(mask), 0u));
}

__device__ __forceinline__ uint64_t bcast64(uint64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(x));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(x >> 32));
  return (uint64_t(hi) << 32) | lo;
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// ---------------------------------------------------------------------------
// the persistent transport kernel
//   kMode: kForward (hit map, optional gradient tallies) or kBackward (replay)
//
// Every lane is EMPTY (no photon), TRAVERSING (searching the closest hit of
// its photon's current step) or WAITING (hit found, interaction pending).
// Each loop iteration every traversing lane takes one micro-step of its BVH
// search: a pop if it holds nothing, one triangle test if it holds a leaf, a
// second pop if that emptied its hands, one node visit if it holds a node.  When
// at least `wave_batch` lanes of the wave are not traversing, the wave runs one
// combined phase for all of them: the interaction of the waiting lanes (and
// the tallies of photons that end), the refill of empty lanes from the photon
// pool, and the start of the next step (free paths, ray set-up).  Lanes thus
// never wait for the slowest search of the wave, and the long, branchy
// interaction code runs once for many lanes instead of once per step.
// ---------------------------------------------------------------------------
enum : int32_t { kEmpty = 0, kTraversing = 1, kWaiting = 2 };

// Five waves per SIMD (at most 96 VGPRs): the lane state of the search and the
// photon fits without spilling; six or more waves force spills that cost more
// than the extra latency hiding gains.
constexpr int kRefillMin = 4;  // empty lanes before a wave refills them

// kOffsets: the launch's sources are POINTS with prefix offsets; the refill
// then finds the sources of the ids it hands out with a wave-uniform cursor
// (one scalar binary search per chunk of ids, then a walk over the few
// sources the chunk spans) instead of a binary search per photon.
template <int kMode, bool kGrad, bool kRecords, bool kCount, bool kOffsets>
__global__ void __launch_bounds__(256, 5) propagate_kernel(const LaunchArgs a) {
  extern __shared__ float4 lds[];
  constexpr bool kGradAcc = kGrad || kMode == kBackward;
  constexpr bool kFwd = kMode != kBackward;
  constexpr bool kTally = kMode == kForwardTally;
  // LDS: the block tallies (kForwardTally launches) from address 0, a
  // constant base, so no register holds their address through the loop: the
  // hit map first (per cell an int32 hit count, or with gradients 4 FP64
  // scores followed by the hit count, 40 bytes), then the loss table and the
  // arrival-time histogram at the byte offsets the host chose (negative: that
  // table goes straight to device memory); the staged BVH levels from
  // node_lds (the tallies' size, a multiple of 128; 0 without tallies), the
  // traversal-stack windows and the counting mode's counters.
  constexpr int32_t kTallyStride = kGrad ? 40 : 4;
  constexpr int32_t kTallyHitOffset = kGrad ? 32 : 0;
  char* const tally = reinterpret_cast<char*>(lds);
  const uint32_t node_lds = kTally ? uint32_t(a.tally_bytes) : 0u;
  float4* lds_nodes = lds + node_lds / 16;
  int32_t* stack_base = reinterpret_cast<int32_t*>(lds_nodes + a.n_lds_nodes * 8);
  unsigned long long* blk_stats =
      reinterpret_cast<unsigned long long*>(stack_base + a.stack_lds * blockDim.x);
  // event caches (offsets variants): this wave's rows after the counters
  constexpr bool kEventCache = kOffsets && kFwd && !kTally;
  int32_t* const ecache = reinterpret_cast<int32_t*>(blk_stats + kStatsWords) +
                          (threadIdx.x >> 6) * (kEventCacheSlots * 64);
  const float4* gn = reinterpret_cast<const float4*>(a.nodes);
  for (int32_t i = threadIdx.x; i < a.n_lds_nodes * 8; i += blockDim.x) lds_nodes[i] = gn[i];
  if (kCount)
    for (int32_t i = threadIdx.x; i < kStatsWords; i += blockDim.x) blk_stats[i] = 0ull;
  if (kTally)
    for (int32_t i = threadIdx.x; i < a.tally_bytes / 4; i += blockDim.x)
      reinterpret_cast<int32_t*>(tally)[i] = 0;
  __syncthreads();
  const int64_t gtid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  lds_i32* const stack_bottom = (lds_i32*)(stack_base) +
                                (threadIdx.x >> 6) * (a.stack_lds * 64) + (threadIdx.x & 63);
  LaneStack stack{stack_bottom, stack_bottom, 256 * (a.stack_lds - 4), a.stack_overflow + gtid,
                  int64_t(gridDim.x) * blockDim.x, a.stack_total, 0};
  const uint32_t lane = lane_rank(~0ull);
  const uint32_t batch_trigger = 64u - uint32_t(a.wave_batch);  // run the phase at <= this

  Photon p;
  int32_t state = kEmpty;
  int64_t idx = 0;
  uint64_t pid = 0;
  uint64_t pool_next = 0, pool_end = 0;
  // kOffsets: a source at or before that of photon pool_next, and the first
  // photon of the source after it (the largest int64 if there is none)
  int64_t cur_src = 0, cur_next = 0;
  bool exhausted = false;
  // event cache: the events of the two rows (-1: none), which row was
  // assigned last, and whether the launch's big chunks are used up
  int64_t erow0 = -1, erow1 = -1;
  int32_t elast = 1;
  bool big_done = false;
  if (kEventCache && a.event_cache) {
    ecache[threadIdx.x & 63] = 0;
    ecache[64 + (threadIdx.x & 63)] = 0;
  }
  Counters cnt{0u, 0u, 0u, 0u};
  uint32_t n_steps = 0;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  // search state of the current step
  StepDraw sd{0.f, 0.f, 0.f};
  Best b{0.f, -1, -1};
  RayW ray;
  f3 inv{0.f, 0.f, 0.f}, oi{0.f, 0.f, 0.f};
  int32_t node = -1, leaf = -1;

  unsigned long long cyc_phase = 0, cyc_search = 0, n_phases = 0;
  while (true) {
    const uint32_t n_trav = uint32_t(__popcll(__ballot(state == kTraversing)));
    unsigned long long t_mark = 0;
    if (kCount) t_mark = clock64();
    if (n_trav <= batch_trigger) {
      if (kCount) n_phases++;
      __builtin_amdgcn_s_setprio(0);
      // ---- interaction of the waiting lanes ----
      bool start = false;  // lanes that begin a new step in this phase
      if (state == kWaiting) {
        state = kTraversing;  // a new step follows unless the photon ends
        start = true;
        if (finish_step<kGradAcc>(p, a, pid, sd, b)) {
          start = false;
          state = kEmpty;
          const int32_t fl = p.flag & 0xff;
          if (fl == F_DETECT) {
            const int64_t cell = int64_t(p.event) * a.n_channels + a.channel_of_sensor[p.sensor];
            // score-function weights of the detected path, evaluated in FP64 (the
            // Rayleigh-length score is a difference of two large terms)
            double sc[4] = {0.0, 0.0, 0.0, 0.0};
            if (kGradAcc) {
              if (a.grad_material >= 0) {
                const DevMaterial gm = a.mats[a.grad_material];
                const double L = p.path_len, la = gm.abs_len, lr = gm.ray_len;
                const double s0 = L / (la * la);
                const double s1 = L / (lr * lr) - double(p.n_sca) / lr;
                sc[0] = isfinite(s0) ? s0 : 0.0;
                sc[1] = isfinite(s1) ? s1 : 0.0;
              }
              sc[2] = p.sum_inv_r;
              sc[3] = p.sum_inv_t;
            }
            if (kFwd) {
              if (kTally && a.tally_cells > 0) {
                // few cells that every workgroup hits: pre-summed in LDS and
                // flushed once per workgroup at exit
                char* const t = tally + int32_t(cell) * kTallyStride;
                if (a.hit_map) atomicAdd(reinterpret_cast<int32_t*>(t + kTallyHitOffset), 1);
                if (kGrad && a.grad) {
#pragma unroll
                  for (int q = 0; q < 4; ++q) atomicAdd(reinterpret_cast<double*>(t) + q, sc[q]);
                }
              } else if (kEventCache && a.event_cache) {
                // the event's row in this wave's LDS cache, or device memory
                const int32_t ch = int32_t(cell - int64_t(p.event) * a.n_channels);
                if (p.event == erow0) atomicAdd(ecache + ch, 1);
                else if (p.event == erow1) atomicAdd(ecache + 64 + ch, 1);
                else atomicAdd(a.hit_map + cell, 1);
              } else if (a.hit_map) {
                atomicAdd(a.hit_map + cell, 1);
              }
              if (a.time_hist) {
                // arrival time bin; the last bin is open-ended (also NaN lands there)
                const float f = p.time * a.time_inv_bin;
                const int32_t bin = f < float(a.n_time_bins - 1) ? int32_t(fmaxf(f, 0.0f))
                                                                 : a.n_time_bins - 1;
                if (kTally && a.lds_time_off >= 0)
                  atomicAdd(reinterpret_cast<int32_t*>(tally + a.lds_time_off) +
                                p.event * a.n_time_bins + bin, 1);
                else
                  atomicAdd(a.time_hist + int64_t(p.event) * a.n_time_bins + bin, 1);
              }
              if ((!kTally || a.tally_cells == 0) && kGrad && a.grad) {
#pragma unroll
                for (int q = 0; q < 4; ++q) atomicAdd(a.grad + cell * 4 + q, sc[q]);
              }
            } else {
              const double w = double(a.grad_hits[cell]);
#pragma unroll
              for (int q = 0; q < 4; ++q) acc[q] += w * sc[q];
            }
          }
          if (kFwd && a.loss) {
            // where the photon ended: the group of its last triangle for the
            // surface terminals, else the material it was in
            const bool on_surface = fl >= F_DETECT && fl <= F_SURFACE_ABSORB && p.last_tri >= 0;
            const int64_t row = on_surface ? int64_t(a.tri_group[p.last_tri])
                                           : int64_t(a.n_groups) + p.medium;
            if (kTally && a.lds_loss_off >= 0)
              atomicAdd(reinterpret_cast<unsigned long long*>(tally + a.lds_loss_off) + row * 8 + fl,
                        1ull);
            else
              atomicAdd(a.loss + row * 8 + fl, 1ull);
          }
          if (kRecords) {
            xp_photon_record& rec = a.records[idx];
            rec.flag = p.flag; rec.last_tri = p.last_tri; rec.sensor = p.sensor; rec.steps = p.steps;
            rec.event = p.event; rec.medium = p.medium; rec.n_scatter = p.n_sca; rec.reserved = 0;
            rec.pos[0] = p.pos.x; rec.pos[1] = p.pos.y; rec.pos[2] = p.pos.z; rec.time = p.time;
            rec.dir[0] = p.dir.x; rec.dir[1] = p.dir.y; rec.dir[2] = p.dir.z;
            rec.path_len = p.path_len;
            rec.pol[0] = p.pol.x; rec.pol[1] = p.pol.y; rec.pol[2] = p.pol.z;
            rec.sum_inv_r = p.sum_inv_r;
            rec.sum_inv_t = p.sum_inv_t; rec.wavelength = p.wavelength;
            rec.pad[0] = rec.pad[1] = 0.0f;
          }
          if (kCount) {
            atomicAdd(&blk_stats[fl], 1ull);
            if (p.flag & F_GEOM) atomicAdd(&blk_stats[8], 1ull);
          }
        }
      }
      // ---- refill empty lanes from the photon pool (wave-uniform control flow) ----
      // Emission costs the whole wave its code path, so a wave refills once at
      // least kRefillMin of its lanes are empty (all of them, when nothing else
      // is left to run).
      uint64_t dead = __ballot(state == kEmpty);
      if (__popcll(dead) < kRefillMin) dead = 0ull;
      while (dead != 0ull && !exhausted) {
        if (pool_next >= pool_end) {
          uint64_t base = 0, end = 0;
          bool got = false;
          if (kEventCache && a.event_cache) {
            // chunks of kBigChunk ids first (work counter's low half), then
            // the launch's chunks after them (its high half)
            if (!big_done) {
              uint64_t c = 0;
              if (lane == 0) c = atomicAdd(a.work_counter, 1ull);
              c = bcast64(c) & 0xffffffffull;
              if (c < uint64_t(a.n_big_chunks)) {
                base = c * uint64_t(kBigChunk);
                end = base + uint64_t(kBigChunk);
                got = true;
              } else {
                big_done = true;
              }
            }
            if (!got) {
              uint64_t c = 0;
              if (lane == 0) c = atomicAdd(a.work_counter, 1ull << 32);
              c = bcast64(c) >> 32;
              base = uint64_t(a.n_big_chunks) * uint64_t(kBigChunk) + c * uint64_t(a.chunk);
            }
          } else {
            if (lane == 0) base = atomicAdd(a.work_counter, (unsigned long long)a.chunk);
            base = bcast64(base);
          }
          if (!got) {
            if (base >= uint64_t(a.n_photons)) {
              exhausted = true;
              break;
            }
            end = min(base + uint64_t(a.chunk), uint64_t(a.n_photons));
          }
          pool_next = base;
          pool_end = end;
          if (kOffsets) {
            cur_src = wave_source_of(a, int64_t(base), lane);
            cur_next = cur_src + 1 < a.n_sources ? uniform64(a.offsets[cur_src + 1]) : INT64_MAX;
            if (kEventCache && a.event_cache && cur_src != erow0 && cur_src != erow1) {
              // the chunk's first event takes the row assigned longer ago: its
              // sums go to device memory (photons of that event still in
              // flight add there directly)
              const int32_t r = 1 - elast;
              const int64_t old = r == 0 ? erow0 : erow1;
              int32_t* row = ecache + r * 64;
              if (old >= 0 && int32_t(lane) < a.n_channels) {
                const int32_t v = row[lane];
                if (v != 0) atomicAdd(a.hit_map + old * a.n_channels + lane, v);
              }
              row[lane] = 0;
              if (r == 0) erow0 = cur_src; else erow1 = cur_src;
              elast = r;
            }
          }
        }
        const uint64_t avail = pool_end - pool_next;
        const uint32_t rank = lane_rank(dead);
        const uint64_t ndead = uint64_t(__popcll(dead));
        const uint64_t ntake = ndead < avail ? ndead : avail;
        int64_t src = -1;
        if (kOffsets) {
          // sources of ids pool_next .. last: walk the offsets forward from the
          // cursor (wave-uniform loads); each lane keeps the last source that
          // starts at or before its id, as the binary search would find
          const int64_t mine = int64_t(pool_next) + int64_t(rank);
          const int64_t last = uniform64(int64_t(pool_next + ntake) - 1);
          const int64_t n_src = uniform64(a.n_sources);
          int64_t s = uniform64(cur_src), next_start = uniform64(cur_next);
          src = s;
          while (next_start <= last) {  // ids up to `last` reach source s + 1
            ++s;
            if (mine >= next_start) src = s;
            next_start = s + 1 < n_src ? uniform64(a.offsets[s + 1]) : INT64_MAX;
          }
          cur_src = s;
          cur_next = next_start;
        }
        if (state == kEmpty && rank < avail) {
          idx = int64_t(pool_next + rank);
          pid = a.pid_base + uint64_t(idx);
          state = kTraversing;
          start = true;
          emit(p, a, idx, pid, src);
        }
        pool_next += ntake;
        dead = __ballot(state == kEmpty);
      }
      if (__ballot(state != kEmpty) == 0ull) break;  // pool exhausted and every lane idle
      // ---- start the next step of the lanes that continue or just got a photon ----
      if (start) {
        sd = begin_step(p, a, pid);
        b = Best{fminf(sd.d_abs, sd.d_sca), -1, -1};
        ray = make_ray(p.pos, p.dir, a.n_tris);
        const float tiny = 1e-30f;
        inv = f3{hw_rcp(fabsf(p.dir.x) > tiny ? p.dir.x : copysignf(tiny, p.dir.x)),
                 hw_rcp(fabsf(p.dir.y) > tiny ? p.dir.y : copysignf(tiny, p.dir.y)),
                 hw_rcp(fabsf(p.dir.z) > tiny ? p.dir.z : copysignf(tiny, p.dir.z))};
        oi = f3{p.pos.x * inv.x, p.pos.y * inv.y, p.pos.z * inv.z};
        node = 0;
        leaf = -1;
        stack.clear();
        if (kCount) n_steps++;
      }
    }
    // Search micro-steps run at a higher wave priority than interaction
    // phases: a micro-step is a short chain of dependent loads, so when both
    // are ready the SIMD issues the search first and lets the phases' long
    // arithmetic fill the wait.  Within the micro-step, the code up to each
    // group of loads (the node, the triangle record) runs at 2, the node
    // visit's arithmetic at 1.
    __builtin_amdgcn_s_setprio(2);
    // ---- one micro-step of every traversing lane's closest-hit search ----
    if (kCount) {
      const unsigned long long t_now = clock64();
      cyc_phase += t_now - t_mark;
      t_mark = t_now;
      cnt.slots++;
    }
    // A micro-step pops an entry if the lane holds nothing, visits at most one
    // node and then tests at most one triangle (the leaf the visit's nearest
    // hit handed over, or one popped or still held): when the wave's lanes are
    // split between the two kinds of work it pays for both either way, so a
    // lane that can do both does.  The closest hit does not depend on the
    // order in which candidates are tested.
    if (state == kTraversing) {
      if (kCount) cnt.busy++;
      if (leaf < 0 && node < 0 && stack.sp > 0) {
        const int32_t e = stack.pop();
        if (e >= 0) node = e; else leaf = ~e;
      }
      if (node >= 0) {
        if (!visit_node<kCount>(a.nodes, a.n_lds_nodes, node_lds, inv, oi, b.t, stack, node, leaf,
                                cnt)) {
          b.tri = kTraversalFailed;
          state = kWaiting;
          node = leaf = -1;
        }
      }
      __builtin_amdgcn_s_setprio(2);
      if (leaf >= 0) {
        // one triangle per micro-step: the packed leaf advances to its next triangle
        if (kCount) cnt.tris++;
        test_triangle(a.tris, leaf >> 3, ray, a.eps, p.last_tri, b);
        // next triangle of the leaf: first + 1, count - 1 (leaf + 7), or done
        leaf = (leaf & 7) != 0 ? leaf + 7 : -1;
      }
      // search complete: b holds the closest hit (or none)
      if (state == kTraversing && leaf < 0 && node < 0 && stack.sp == 0) state = kWaiting;
    }
    if (kCount) cyc_search += clock64() - t_mark;
  }

  // ---- the wave's event-cache rows to device memory ----
  if (kEventCache && a.event_cache && int32_t(lane) < a.n_channels) {
    const int32_t v0 = ecache[lane], v1 = ecache[64 + lane];
    if (erow0 >= 0 && v0 != 0) atomicAdd(a.hit_map + erow0 * a.n_channels + lane, v0);
    if (erow1 >= 0 && v1 != 0) atomicAdd(a.hit_map + erow1 * a.n_channels + lane, v1);
  }

  // ---- block tallies to global memory (every wave of the block has left the loop) ----
  if (kTally) {
    __syncthreads();
    if (a.lds_time_off >= 0) {
      const int32_t* h = reinterpret_cast<const int32_t*>(tally + a.lds_time_off);
      for (int32_t i = threadIdx.x; i < a.n_time_cells; i += blockDim.x)
        if (h[i] != 0) atomicAdd(a.time_hist + i, h[i]);
    }
    if (a.lds_loss_off >= 0) {
      const unsigned long long* l = reinterpret_cast<const unsigned long long*>(tally + a.lds_loss_off);
      for (int32_t i = threadIdx.x; i < a.n_loss_cells; i += blockDim.x)
        if (l[i] != 0ull) atomicAdd(a.loss + i, l[i]);
    }
    for (int32_t i = threadIdx.x; i < a.tally_cells; i += blockDim.x) {
      const char* t = tally + i * kTallyStride;
      const int32_t h = *reinterpret_cast<const int32_t*>(t + kTallyHitOffset);
      if (a.hit_map && h != 0) atomicAdd(a.hit_map + i, h);
      if (kGrad && a.grad) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double v = reinterpret_cast<const double*>(t)[q];
          if (v != 0.0) atomicAdd(a.grad + int64_t(i) * 4 + q, v);
        }
      }
    }
  }

  // ---- per-wave reductions at exit ----
  if (kMode == kBackward) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double s = wave_sum(acc[q]);
      if (lane == 0 && s != 0.0) atomicAdd(a.grad_params + q, s);
    }
  }
  if (kCount) {
    const unsigned long long s9 = wave_sum_u64(n_steps);
    const unsigned long long s10 = wave_sum_u64(cnt.nodes);
    const unsigned long long s11 = wave_sum_u64(cnt.tris);
    const unsigned long long s12 = wave_sum_u64(cnt.slots);
    const unsigned long long s13 = wave_sum_u64(cnt.busy);
    if (lane == 0) {
      atomicAdd(&blk_stats[9], s9);
      atomicAdd(&blk_stats[10], s10);
      atomicAdd(&blk_stats[11], s11);
      atomicAdd(&blk_stats[12], s12);
      atomicAdd(&blk_stats[13], s13);
      atomicAdd(&blk_stats[15], n_phases);
      atomicAdd(&blk_stats[16], cyc_phase);
      atomicAdd(&blk_stats[17], cyc_search);
    }
    __syncthreads();
    if (threadIdx.x < 18 && a.stats) atomicAdd(a.stats + threadIdx.x, blk_stats[threadIdx.x]);
  }
}

}  // namespace
}  // namespace xp

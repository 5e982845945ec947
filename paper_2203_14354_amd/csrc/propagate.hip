// propagate.hip -- host launchers of the transport kernels, the kernel
// variants without LDS tallies, and the small kernels behind the test hooks
// (closest hit, emission sampling, reflectance, arrival-time quantiles,
// streaming-read probe).  The transport itself is in transport.h.
#include <mutex>

#include "transport.h"

namespace xp {

// Scratch of xp_propagate_static, a file-scope device array that every device
// the module runs on holds until the process ends, so that the entry point
// needs no allocation.  Host code never passes the array's name to a kernel
// (on the host it is only a stand-in for the symbol); it passes the device
// address hipGetSymbolAddress returns, kept per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kScratchDevices = 64;
std::mutex scratch_mutex;
void* scratch_address[kScratchDevices] = {};
}  // namespace

hipError_t scratch_init(int device) {
  if (device < 0 || device >= kScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mutex);
  if (scratch_address[device] != nullptr) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (p == nullptr) return hipErrorInvalidSymbol;
  scratch_address[device] = p;
  return hipSuccess;
}

void* scratch_base(int device) {
  if (device < 0 || device >= kScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lock(scratch_mutex);
  return scratch_address[device];
}

namespace {

__global__ void reset_kernel(unsigned long long* counter) { *counter = 0ull; }

// closest hit for a batch of rays (test hook)
__global__ void __launch_bounds__(64) closest_hit_kernel(const Node4* nodes, const TriRec* tris,
                                                         int32_t n_tris, int32_t stack_depth,
                                                         int64_t n, const float* orig,
                                                         const float* dir, const int32_t* skip,
                                                         float tmin, float tmax, int32_t brute,
                                                         int32_t* out_tri, float* out_t) {
  extern __shared__ float4 lds[];
  // the whole worst-case stack in LDS: stack_depth is at least the bound
  // plus the four slots a visit reserves; with the usable depth capped at
  // stack_depth - 4 the window never spills (no overflow array)
  lds_i32* const bottom = (lds_i32*)(reinterpret_cast<int32_t*>(lds)) + threadIdx.x;  // one wave per block
  LaneStack stack{bottom, bottom, 256 * (stack_depth - 4), nullptr, 0, stack_depth - 4, 0};
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const f3 o{orig[3 * i], orig[3 * i + 1], orig[3 * i + 2]};
  const f3 d{dir[3 * i], dir[3 * i + 1], dir[3 * i + 2]};
  const int32_t sk = skip ? skip[i] : -1;
  Best b{tmax, -1, -1};
  Counters c{0u, 0u, 0u, 0u};
  bool ok = true;
  if (brute) {
    const RayW r = make_ray(o, d, n_tris);
    for (int32_t k = 0; k < n_tris; ++k) test_triangle(tris, k, r, tmin, sk, b);
  } else {
    // no node is staged in LDS (n_lds = 0): the LDS holds the stack windows
    ok = traverse<false>(nodes, 0, tris, n_tris, stack, o, d, tmin, sk, b, c);
  }
  out_tri[i] = ok ? b.tri : -2;
  out_t[i] = b.tri >= 0 ? b.t : kInfF;
}

// streaming read of a buffer, `passes` times with a grid stride (bandwidth
// probe).  Each thread keeps four independent 16-byte loads in flight, so that
// the chip holds enough outstanding requests to reach the bandwidth of the
// level the buffer lives in rather than its latency bound.
__global__ void __launch_bounds__(256) stream_read_kernel(const float4* __restrict__ buf, int64_t n,
                                                          int32_t passes, float* out) {
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  float acc0 = 0.0f, acc1 = 0.0f, acc2 = 0.0f, acc3 = 0.0f;
  for (int32_t k = 0; k < passes; ++k) {
    int64_t i = gid;
    for (; i + 3 * stride < n; i += 4 * stride) {
      const float4 v0 = buf[i], v1 = buf[i + stride], v2 = buf[i + 2 * stride],
                   v3 = buf[i + 3 * stride];
      acc0 += (v0.x + v0.y) + (v0.z + v0.w);
      acc1 += (v1.x + v1.y) + (v1.z + v1.w);
      acc2 += (v2.x + v2.y) + (v2.z + v2.w);
      acc3 += (v3.x + v3.y) + (v3.z + v3.w);
    }
    for (; i < n; i += stride) {
      const float4 v = buf[i];
      acc0 += (v.x + v.y) + (v.z + v.w);
    }
  }
  out[gid] = (acc0 + acc1) + (acc2 + acc3);
}

// VALU issue probe (calibrates the SQ instruction and cycle counters against
// a known instruction count): every thread runs `iters` iterations of 64
// steps on eight independent chains, with scalar loop control.  Kinds, with
// the VALU instructions per step:
//   0 FP32 multiply-add (one);  1 FP32 reciprocal, a transcendental (one);
//   2 32-bit integer xor then add (two);
//   3 an FP32 multiply-add and an independent integer xor and add (three);
//   4 an FP32 multiply-add and an independent FP32 reciprocal (two);
//   5 a 32 x 32 -> 64-bit integer multiply-add (Philox's product) and a move
//     of its high half (two).
// Kinds 3 and 4 mix instruction types within a wave, the case in which the
// counters of the transport kernel show two VALU instructions issued in one
// cycle group.
template <int kKind>
__global__ void __launch_bounds__(256) valu_probe_kernel(float m, float c, int32_t iters,
                                                         float* out) {
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  float a[8], b[8];
  uint32_t q[8];
  uint64_t w[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    a[j] = float(threadIdx.x) * 1e-3f + float(j);
    b[j] = 1.0f + float(j);
    q[j] = threadIdx.x + uint32_t(j);
    w[j] = uint64_t(threadIdx.x) * 3u + uint64_t(j);
  }
  const uint32_t mb = __float_as_uint(m), cb = __float_as_uint(c);
  for (int32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if (kKind == 0 || kKind == 3 || kKind == 4) a[j] = fmaf(a[j], m, c);
        if (kKind == 1 || kKind == 4) b[j] = __builtin_amdgcn_rcpf(b[j]);
        if (kKind == 2 || kKind == 3) q[j] = (q[j] ^ mb) + cb;
        if (kKind == 5) w[j] = uint64_t(uint32_t(w[j])) * mb + (w[j] >> 32);
      }
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    if (kKind == 0) s += a[j];
    if (kKind == 1) s += b[j];
    if (kKind == 2) s += float(q[j]);
    if (kKind == 3) s += a[j] + float(q[j]);
    if (kKind == 4) s += a[j] + b[j];
    if (kKind == 5) s += float(uint32_t(w[j]));
  }
  out[gid] = s;
}

// emission wavelengths with the transport's random-number schedule (test hook)
__global__ void wavelength_kernel(uint32_t s0, uint32_t s1, uint64_t pid0, int64_t n, float mean,
                                  float sigma, float* out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = emission_wavelength(s0, s1, pid0 + uint64_t(i), mean, sigma);
}

// |r_s|^2, |r_p|^2 of a complex-index / thin-film surface (test hook)
__global__ void reflectance_kernel(int32_t model, float n1, float n_re, float n_im, float film_n,
                                   float two_pi_d, float lam, int64_t n, const float* cos_i,
                                   float* out_rs, float* out_rp) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  cf rs, rp;
  film_reflection(model, n1, cos_i[i], n_re, n_im, film_n, two_pi_d, lam, rs, rp);
  out_rs[i] = c_norm(rs);
  out_rp[i] = c_norm(rp);
}

// emission times with the transport's random-number schedule (test hook)
__global__ void emission_time_kernel(uint32_t s0, uint32_t s1, uint64_t pid0, int64_t n,
                                     float tau_singlet, float tau_triplet, float singlet_fraction,
                                     float* out_t, int32_t* out_singlet) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  bool singlet;
  out_t[i] = emission_time(s0, s1, pid0 + uint64_t(i), tau_singlet, tau_triplet,
                           singlet_fraction, singlet);
  if (out_singlet) out_singlet[i] = singlet ? 1 : 0;
}

// Quantile q of each event's arrival-time histogram: the first bin where the
// cumulative count reaches q * total, interpolated linearly inside it.  One
// thread per event; counts summed in 64-bit integers, the target in FP64.
__global__ void time_quantile_kernel(const int32_t* hist, int64_t n_events, int32_t n_bins,
                                     float bin_ns, float q, float* out) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n_events) return;
  const int32_t* h = hist + e * n_bins;
  int64_t total = 0;
  for (int32_t b = 0; b < n_bins; ++b) total += h[b];
  if (total == 0) {
    out[e] = __builtin_nanf("");
    return;
  }
  const double target = double(q) * double(total);
  int64_t cum = 0;
  float res = kInfF;
  for (int32_t b = 0; b < n_bins; ++b) {
    const int64_t c = h[b];
    if (c > 0 && double(cum + c) >= target) {
      res = b == n_bins - 1 ? kInfF
                            : float((double(b) + (target - double(cum)) / double(c)) * double(bin_ns));
      break;
    }
    cum += c;
  }
  out[e] = res;
}

// samplers with the transport's random-number schedule (test hook)
__global__ void sample_kernel(int32_t kind, uint32_t s0, uint32_t s1, uint64_t pid0, int64_t n,
                              const float* in_dir, const float* in_pol, float cyl_r, float zlo,
                              float zhi, float* out_dir, float* out_pol) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t pid = pid0 + uint64_t(i);
  Photon p;
  p.pos = p.dir = p.pol = f3{0.f, 0.f, 0.f};
  if (kind == 0) {
    const R4 r = draw(s0, s1, pid, 0u, 0u);
    p.dir = isotropic(r.u0, r.u1);
    p.pol = random_polarization(p.dir, r.u2);
  } else if (kind == 1) {
    lambertian(p, f3{in_dir[3 * i], in_dir[3 * i + 1], in_dir[3 * i + 2]}, draw(s0, s1, pid, 1u, 1u));
  } else if (kind == 2) {
    p.dir = f3{in_dir[3 * i], in_dir[3 * i + 1], in_dir[3 * i + 2]};
    p.pol = f3{in_pol[3 * i], in_pol[3 * i + 1], in_pol[3 * i + 2]};
    rayleigh(p, s0, s1, pid, 1u, draw(s0, s1, pid, 1u, 2u));
  } else {
    p.dir = cylinder_point(s0, s1, pid, cyl_r, zlo, zhi);  // the transport's emission code
  }
  out_dir[3 * i] = p.dir.x; out_dir[3 * i + 1] = p.dir.y; out_dir[3 * i + 2] = p.dir.z;
  out_pol[3 * i] = p.pol.x; out_pol[3 * i + 1] = p.pol.y; out_pol[3 * i + 2] = p.pol.z;
}

template <int kMode, bool kGrad, bool kRecords, bool kCount, bool kOffsets = false>
hipError_t launch_one(const LaunchArgs& a, int block, int grid, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL((propagate_kernel<kMode, kGrad, kRecords, kCount, kOffsets>), dim3(grid),
                     dim3(block), lds, s, a);
  return hipGetLastError();
}

}  // namespace

size_t propagate_lds_bytes(int32_t n_lds_nodes, int32_t stack_lds, int block, size_t tally_bytes) {
  return tally_bytes + size_t(n_lds_nodes) * sizeof(Node4) + size_t(stack_lds) * block * 4 +
         kStatsWords * sizeof(unsigned long long);
}

hipError_t launch_reset(unsigned long long* counter, hipStream_t s) {
  hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(1), 0, s, counter);
  return hipGetLastError();
}

hipError_t launch_propagate(const LaunchArgs& a, int mode, bool grad, bool records, bool count,
                            int block, int grid, hipStream_t s) {
  // block tallies only in the plain forward launch (no records, no counters)
  const bool tally = mode == kForward && a.tally_bytes > 0 && !records && !count;
  const size_t lds = propagate_lds_bytes(a.n_lds_nodes, a.stack_lds, block,
                                         tally ? size_t(a.tally_bytes) : 0) +
                     (a.event_cache ? event_cache_lds_bytes(block) : 0);
  // sources with prefix offsets: the variants with the wave-uniform source
  // cursor (records and counters keep the per-photon search; same results)
  const bool offs = a.src_kind == XP_SRC_POINTS && a.offsets != nullptr;
  if (mode == kBackward) {
    if (records || count || grad) return hipErrorInvalidValue;
    return offs ? launch_one<kBackward, false, false, false, true>(a, block, grid, lds, s)
                : launch_one<kBackward, false, false, false>(a, block, grid, lds, s);
  }
  if (mode != kForward) return hipErrorInvalidValue;
  if (tally) return launch_propagate_tally(a, grad, offs, block, grid, lds, s);
  if (offs && !records && !count)
    return grad ? launch_one<kForward, true, false, false, true>(a, block, grid, lds, s)
                : launch_one<kForward, false, false, false, true>(a, block, grid, lds, s);
  const int key = (grad ? 4 : 0) | (records ? 2 : 0) | (count ? 1 : 0);
  switch (key) {
    case 0: return launch_one<kForward, false, false, false>(a, block, grid, lds, s);
    case 1: return launch_one<kForward, false, false, true>(a, block, grid, lds, s);
    case 2: return launch_one<kForward, false, true, false>(a, block, grid, lds, s);
    case 3: return launch_one<kForward, false, true, true>(a, block, grid, lds, s);
    case 4: return launch_one<kForward, true, false, false>(a, block, grid, lds, s);
    case 5: return launch_one<kForward, true, false, true>(a, block, grid, lds, s);
    case 6: return launch_one<kForward, true, true, false>(a, block, grid, lds, s);
    default: return launch_one<kForward, true, true, true>(a, block, grid, lds, s);
  }
}

hipError_t max_blocks_per_cu(int block, size_t lds_bytes, bool count, bool tally, int* out) {
  if (tally) return max_blocks_per_cu_tally(block, lds_bytes, out);
  if (count)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        out, reinterpret_cast<const void*>(propagate_kernel<kForward, true, true, true, false>),
        block, lds_bytes);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(
      out, reinterpret_cast<const void*>(propagate_kernel<kForward, false, false, false, false>),
      block, lds_bytes);
}

hipError_t launch_emission_time(uint64_t seed, uint64_t pid0, int64_t n, float tau_singlet,
                                float tau_triplet, float singlet_fraction, float* out_t,
                                int32_t* out_singlet, hipStream_t s) {
  const int block = 256;
  const int64_t grid = (n + block - 1) / block;
  hipLaunchKernelGGL(emission_time_kernel, dim3(uint32_t(grid)), dim3(block), 0, s,
                     uint32_t(seed), uint32_t(seed >> 32), pid0, n, tau_singlet, tau_triplet,
                     singlet_fraction, out_t, out_singlet);
  return hipGetLastError();
}

hipError_t launch_stream_read(const void* buf, int64_t n_vec, int32_t passes, int32_t blocks,
                              float* out, hipStream_t s) {
  hipLaunchKernelGGL(stream_read_kernel, dim3(uint32_t(blocks)), dim3(256), 0, s,
                     static_cast<const float4*>(buf), n_vec, passes, out);
  return hipGetLastError();
}

hipError_t launch_valu_probe(int32_t kind, float m, float c, int32_t iters, int32_t blocks,
                             float* out, hipStream_t s) {
  const dim3 grid{uint32_t(blocks)}, block{256u};
  switch (kind) {
    case 0: hipLaunchKernelGGL(valu_probe_kernel<0>, grid, block, 0, s, m, c, iters, out); break;
    case 1: hipLaunchKernelGGL(valu_probe_kernel<1>, grid, block, 0, s, m, c, iters, out); break;
    case 2: hipLaunchKernelGGL(valu_probe_kernel<2>, grid, block, 0, s, m, c, iters, out); break;
    case 3: hipLaunchKernelGGL(valu_probe_kernel<3>, grid, block, 0, s, m, c, iters, out); break;
    case 4: hipLaunchKernelGGL(valu_probe_kernel<4>, grid, block, 0, s, m, c, iters, out); break;
    case 5: hipLaunchKernelGGL(valu_probe_kernel<5>, grid, block, 0, s, m, c, iters, out); break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_wavelength(uint64_t seed, uint64_t pid0, int64_t n, float mean, float sigma,
                             float* out, hipStream_t s) {
  const int block = 256;
  const int64_t grid = (n + block - 1) / block;
  hipLaunchKernelGGL(wavelength_kernel, dim3(uint32_t(grid)), dim3(block), 0, s, uint32_t(seed),
                     uint32_t(seed >> 32), pid0, n, mean, sigma, out);
  return hipGetLastError();
}

hipError_t launch_reflectance(int32_t model, float n1, float n_re, float n_im, float film_n,
                              float two_pi_d, float lambda, int64_t n, const float* cos_i,
                              float* out_rs, float* out_rp, hipStream_t s) {
  const int block = 256;
  const int64_t grid = (n + block - 1) / block;
  hipLaunchKernelGGL(reflectance_kernel, dim3(uint32_t(grid)), dim3(block), 0, s, model, n1, n_re,
                     n_im, film_n, two_pi_d, lambda, n, cos_i, out_rs, out_rp);
  return hipGetLastError();
}

hipError_t launch_time_quantile(const int32_t* hist, int64_t n_events, int32_t n_bins,
                                float bin_ns, float q, float* out, hipStream_t s) {
  const int block = 256;
  const int64_t grid = (n_events + block - 1) / block;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(time_quantile_kernel, dim3(uint32_t(grid)), dim3(block), 0, s, hist,
                     n_events, n_bins, bin_ns, q, out);
  return hipGetLastError();
}

hipError_t launch_closest_hit(const Node4* nodes, const TriRec* tris, int32_t n_tris,
                              int32_t stack_depth, int64_t n, const float* orig, const float* dir,
                              const int32_t* skip, float tmin, float tmax, int32_t brute,
                              int32_t* out_tri, float* out_t, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int block = 64;
  const int64_t grid = (n + block - 1) / block;
  const size_t lds = size_t(stack_depth) * block * 4;
  hipLaunchKernelGGL(closest_hit_kernel, dim3(unsigned(grid)), dim3(block), lds, s, nodes, tris,
                     n_tris, stack_depth, n, orig, dir, skip, tmin, tmax, brute, out_tri, out_t);
  return hipGetLastError();
}

hipError_t launch_sample(int32_t kind, uint64_t seed, uint64_t pid0, int64_t n, const float* in_dir,
                         const float* in_pol, float cyl_r, float zlo, float zhi, float* out_dir,
                         float* out_pol, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int block = 256;
  const int64_t grid = (n + block - 1) / block;
  hipLaunchKernelGGL(sample_kernel, dim3(unsigned(grid)), dim3(block), 0, s, kind, uint32_t(seed),
                     uint32_t(seed >> 32), pid0, n, in_dir, in_pol, cyl_r, zlo, zhi, out_dir,
                     out_pol);
  return hipGetLastError();
}

}  // namespace xp

// grca_kernels.hip -- HIP kernels of the emitter-centric caster for gfx950
// (wave64, CDNA4).  No MFMA: nothing on this path is a dense contraction.
//
// Per cast:
//   init_kernel      keys = KEY_INIT, counters cleared            (bookend pass)
//   bounds_kernel    per triangle, per observing sensor: range prefilter,
//                    elevation extent -> channel span, azimuth arc -> ray span,
//                    small/large classification, wave-aggregated queue append
//   expand_kernel    persistent: per large record, per channel, the exact
//                    azimuth arc(s) of the channel cone inside the triangle
//                    -> per-channel row items
//   isect_kernel     persistent, candidate-balanced tickets: FP64 statics per
//                    item, flattened candidates, FP32 ray test, 64-bit atomic
//                    minimum on packed keys
//   resolve_kernel   keys -> (distance, triangle id)                (bookend)
// plus the all-pairs reference, the pose (dynamic geometry) kernel and the
// sensor-table builder.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <math.h>
#include <stdint.h>

#include "grca_device.hpp"
#include "grca_launch.hpp"

namespace grca {

constexpr double TWO_PI = 6.283185307179586476925286766559;
constexpr float TWO_PI_F = 6.28318530717958647692f;
constexpr float PI_F = 3.14159265358979323846f;

// Conservative margins of the FP32 bounds pass, each at least ten times the
// FP32 error it covers (local frame, bounded atan2, table rounding):
// elevation margin in sine units, azimuth margin in radians, and the
// |sin(elevation)| beyond which the azimuth arc is taken as the full turn.
constexpr float ETA_SIN = 4e-6f;
constexpr float MARGIN_AZ = 2e-5f;
constexpr float MARGIN_AZ_POLE = 1e-6f;
constexpr float S_POLE = 0.9999f;
// Angular margin (sine) of the per-channel arcs of the large class.
constexpr double SIN_M = 4e-6;
// Candidate pairs one queue shard may hold (item candidate starts are 32-bit;
// staying below 2^31 keeps the intersection tickets from wrapping).
constexpr uint32_t CAND_LIMIT = 0x80000000u;

__device__ inline uint32_t lane_id() { return __lane_id(); }

// Lane 0's value, as a wave-uniform (scalar) value (every lane active).
__device__ inline uint32_t first_lane(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ inline float first_lane(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ inline unsigned long long first_lane(unsigned long long v) {
  return (unsigned long long)first_lane((uint32_t)v) |
         ((unsigned long long)first_lane((uint32_t)(v >> 32)) << 32);
}

// Index of the calling wave within its block, as a wave-uniform (scalar)
// value: everything derived from it (tile, scene, sensor loop) then stays in
// scalar registers and scalar loads.
// Global load at a 32-bit byte offset from a wave-uniform base: the address
// is the scalar base plus the zero-extended offset, with no 64-bit vector
// arithmetic.
template <typename T>
__device__ inline T gload(const T* base, uint32_t byte_off) {
  typedef const T __attribute__((address_space(1))) GT;
  typedef const char __attribute__((address_space(1))) GC;
  return *(GT*)((GC*)base + byte_off);
}

// A vertex (x, y, z; the fourth component is padding) at a 32-bit byte offset.
__device__ inline float4 gload_v(const float4* base, uint32_t byte_off) {
  typedef float v4f __attribute__((ext_vector_type(4)));
  typedef const v4f __attribute__((address_space(1))) GT;
  typedef const char __attribute__((address_space(1))) GC;
  const v4f q = *(GT*)((GC*)base + byte_off);
  return make_float4(q.x, q.y, q.z, q.w);
}

// A triangle's three vertex indices (12 bytes at a 4-byte aligned offset), in
// one load.
struct Tri3 {
  uint32_t a, b, c;
};
__device__ inline Tri3 gload_tri(const uint32_t* base, uint32_t byte_off) {
  typedef uint32_t v3u __attribute__((ext_vector_type(3)));
  typedef const v3u __attribute__((address_space(1))) GT;
  typedef const char __attribute__((address_space(1))) GC;
  const v3u q = *(GT*)((GC*)base + byte_off);
  return Tri3{q.x, q.y, q.z};
}

__device__ inline float2 gload_f2(const float2* base, uint32_t byte_off) {
  const unsigned long long v = gload(reinterpret_cast<const unsigned long long*>(base), byte_off);
  return make_float2(__uint_as_float((uint32_t)v), __uint_as_float((uint32_t)(v >> 32)));
}

// Lane l's value of a double (wave-uniform result).
__device__ inline double lane_f64(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Number of lanes below this one whose bit is set in mask m (v_mbcnt).
__device__ inline uint32_t rank_in(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ inline uint32_t wave_id() {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Inclusive prefix sum over the wave by DPP: row shifts within each row of
// 16 lanes (a lane with no source reads 0), then the row totals broadcast
// to the following rows.  No LDS round trips.
__device__ inline uint32_t wave_incl_scan(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x111, 0xf, 0xf, true);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x112, 0xf, 0xf, true);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x114, 0xf, 0xf, true);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x118, 0xf, 0xf, true);  // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}
// The value of lane 63, as a wave-uniform value.
__device__ inline uint32_t last_lane(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Append one record per lane with `want` set, one atomic per wave.
__device__ inline void wave_push(bool want, const Item& rec, Item* q, uint32_t cap,
                                 uint32_t* counter, uint32_t* overflow, uint32_t ovf_bit,
                                 uint32_t* stat) {
  const unsigned long long mask = __ballot(want);
  if (mask == 0ull) return;
  const uint32_t n = (uint32_t)__popcll(mask);
  const int leader = __ffsll((long long)mask) - 1;
  uint32_t base = 0;
  if ((int)lane_id() == leader) {
    base = atomicAdd(counter, n);
    if (stat) atomicAdd(stat, n);
  }
  base = (uint32_t)__builtin_amdgcn_readlane((int)base, leader);
  if (want) {
    const uint32_t rank = rank_in(mask);
    const uint32_t slot = base + rank;
    if (slot < cap) {
      q[slot] = rec;
    } else {
      atomicOr(overflow, ovf_bit);
    }
  }
}

// ------------------------------------------------------------------ init
static_assert(NSHARD == 64, "the summary reduces one shard per lane of a wave");

__global__ void init_kernel(unsigned long long* __restrict__ keys, uint32_t n,
                            Counters* __restrict__ cnt) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) keys[g] = KEY_INIT;
  // everything but the sticky overflow record
  constexpr uint32_t WORDS = (uint32_t)(__builtin_offsetof(Counters, sticky) / sizeof(uint32_t));
  if (g < WORDS) reinterpret_cast<uint32_t*>(cnt)[g] = 0u;
}

// ------------------------------------------------------------------ bounds
struct Span {
  uint32_t c_from, c_count;
  uint32_t r0_start, r0_count, r1_start, r1_count;
  bool large;
};

// Bin of the sine -> channel lookup for sine x, one bin early: the FP32 bin
// index may round up.
__device__ inline uint32_t chan_bin(const DevSensor& s, float x) {
  const float fb = (x + 1.0f) * (0.5f * (float)s.lut_size);
  const int b = (fb > 0.0f) ? (int)fminf(fb, (float)(s.lut_size - 1)) : 0;
  return b > 0 ? (uint32_t)(b - 1) : 0u;
}

// A bin as one 16-byte load (a field-by-field read under conditions can
// become a chain of dependent loads).
__device__ inline ChanBin load_bin(const ChanBin* p) {
  const uint4 q = *reinterpret_cast<const uint4*>(p);
  return ChanBin{q.x, __uint_as_float(q.y), __uint_as_float(q.z), __uint_as_float(q.w)};
}

// first j with sin_tab[j] >= x (strict = false) or > x (strict = true), from
// the bin's entry e
__device__ inline uint32_t chan_resolve(const DevSensor& s, const ChanBin& e, float x,
                                        bool strict) {
  uint32_t j = e.j;
  if (strict) {
    j += (uint32_t)(e.s0 <= x) + (uint32_t)(e.s1 <= x) + (uint32_t)(e.s2 <= x);
    if (e.s2 <= x)  // channels closer than the bins: walk on
      while (j < s.gamma && s.sin_tab[j] <= x) ++j;
  } else {
    j += (uint32_t)(e.s0 < x) + (uint32_t)(e.s1 < x) + (uint32_t)(e.s2 < x);
    if (e.s2 < x)
      while (j < s.gamma && s.sin_tab[j] < x) ++j;
  }
  return j;
}

__device__ inline uint32_t chan_search(const DevSensor& s, float x, bool strict) {
  return chan_resolve(s, load_bin(s.bins + chan_bin(s, x)), x, strict);
}

// atan2(y, x) in FP32 for the bounds pass, |error| <= 5e-7 rad for mx > 0
// (libm's atan2f is within about 2.4e-7): reduction to t = min(|x|,|y|) /
// max(|x|,|y|) in [0, 1] with the hardware reciprocal, atan(t) = t P(t^2)
// with P of degree 7, then the reflections of the octant.  The coefficients
// were fitted to atan on [0, 1] by least squares reweighted toward the
// minimax (Lawson) error; tests/test_atan_bound.py checks the bound.
__device__ inline float atan_unit(float t) {  // atan(t), t in [0, 1]
  const float u = t * t;
  float p = -0.00405456498f;
  p = fmaf(p, u, 0.0218629558f);
  p = fmaf(p, u, -0.0559123345f);
  p = fmaf(p, u, 0.0964219868f);
  p = fmaf(p, u, -0.139086306f);
  p = fmaf(p, u, 0.199465662f);
  p = fmaf(p, u, -0.333298594f);
  p = fmaf(p, u, 0.999999344f);
  return p * t;
}
__device__ inline float atan2_bounded(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
  const float t = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
  float r = atan_unit(t);
  if (ay > ax) r = 1.57079637f - r;
  if (x < 0.0f) r = 3.14159274f - r;
  return y < 0.0f ? -r : r;
}

// atan(t), t in [0, 1], to 1.8e-6 rad (a 6-term odd polynomial fitted for
// this file): for the sphere tests, whose elevation margin is 3e-5 rad.
__device__ inline float atan_unit_coarse(float t) {
  const float u = t * t;
  float p = -0.0116878422f;
  p = fmaf(p, u, 0.0525693297f);
  p = fmaf(p, u, -0.116357207f);
  p = fmaf(p, u, 0.193514258f);
  p = fmaf(p, u, -0.332618982f);
  p = fmaf(p, u, 0.999977052f);
  return p * t;
}

// atan2 for x >= 0 (the right half-plane: an elevation from a horizontal
// distance), for the sphere tests: atan2_bounded's steps with the coarse
// polynomial, without the reflection for x < 0 and without the guard for
// x = y = 0, which gives NaN here.
__device__ inline float atan2_right(float y, float x) {
  const float ay = fabsf(y);
  const float mx = fmaxf(x, ay), mn = fminf(x, ay);
  float r = atan_unit_coarse(mn * __builtin_amdgcn_rcpf(mx));
  if (ay > x) r = 1.57079637f - r;
  return y < 0.0f ? -r : r;
}

// Ray span of a (triangle, sensor) pair from its vertices in local
// coordinates (x forward, y right): the azimuth arc widened by the FP32
// margins, as one or two ray-index ranges (r0, r1), or the whole turn when
// `full` is set or the arc is too wide.  Returns false when no ray falls in
// it (`full` is set when the whole turn is taken).  `smax_abs` is the
// largest |sine of elevation| of the triangle, which sets the pole margin.
__device__ inline bool ray_span(const float (&x)[3], const float (&y)[3], float smax_abs,
                                bool& full, const DevSensor& s, Span& sp) {
  const uint32_t chi = s.chi;
  sp.r1_start = 0; sp.r1_count = 0;
  if (!full) {
    // Azimuth of vertex 0, and the offsets of vertices 1 and 2 from it.  An
    // offset of tangent t = cross / dot with |t| <= 0.1 lies in
    // [t - |t|^3/3, t + |t|^3/3] (atan's alternating series), so small
    // triangles need one atan2 instead of three; other offsets take the full
    // atan2 difference, wrapped to (-pi, pi].
    const float t0 = atan2_bounded(y[0], x[0]);
    float lo = 0.0f, hi = 0.0f;
#pragma unroll
    for (int k = 1; k < 3; ++k) {
      const float cr = fmaf(x[0], y[k], -(y[0] * x[k]));
      const float dt = fmaf(x[0], x[k], y[0] * y[k]);
      if (dt > 0.0f && fabsf(cr) <= 0.1f * dt) {
        const float t = cr * __builtin_amdgcn_rcpf(dt);
        const float c3 = fabsf(t) * t * t * (1.0f / 3.0f);
        lo = fminf(lo, t - c3);
        hi = fmaxf(hi, t + c3);
      } else {
        float d = atan2_bounded(y[k], x[k]) - t0;
        if (d > PI_F) d -= TWO_PI_F;
        if (d < -PI_F) d += TWO_PI_F;
        lo = fminf(lo, d);
        hi = fmaxf(hi, d);
      }
    }
    if (hi - lo > PI_F - 1e-3f) {
      full = true;
    } else {
      // 1 / max(cos(max |elevation|), 1e-3) by the hardware reciprocal square
      // root (1 ulp suffices for a margin term)
      const float inv_cos = __builtin_amdgcn_rsqf(fmaxf(fmaf(-smax_abs, smax_abs, 1.0f), 1e-6f));
      const float m = MARGIN_AZ + MARGIN_AZ_POLE * inv_cos + s.az_noise;
      float a = t0 + lo - m - s.theta_start;
      a -= TWO_PI_F * floorf(a * (1.0f / TWO_PI_F));
      if (a < 0.0f) a = 0.0f;
      const float w = (hi - lo) + 2.0f * m;
      const float fa = a * s.inv_dtheta;
      const float fb = (a + w) * s.inv_dtheta;
      const int ra = (int)ceilf(fa);
      const int rb = (int)floorf(fb);
      if (s.wrap) {
        int cnt = rb - ra + 1;
        if (cnt <= 0) return false;
        if (cnt > (int)chi) cnt = (int)chi;
        // a lies in [0, 2 pi] up to rounding, so ra lies in [0, chi + 1]
        sp.r0_start = (uint32_t)ra >= chi ? (uint32_t)ra - chi : (uint32_t)ra;
        sp.r0_count = (uint32_t)cnt;
      } else {
        sp.r0_count = 0;
        if (ra <= (int)chi - 1 && rb >= ra) {
          const int e0 = rb < (int)chi - 1 ? rb : (int)chi - 1;
          sp.r0_start = (uint32_t)ra;
          sp.r0_count = (uint32_t)(e0 - ra + 1);
        }
        const float fb2 = (a + w - TWO_PI_F) * s.inv_dtheta;
        if (fb2 >= 0.0f) {
          int e1 = (int)floorf(fb2);
          if (e1 > (int)chi - 1) e1 = (int)chi - 1;
          sp.r1_start = 0;
          sp.r1_count = (uint32_t)(e1 + 1);
          if (sp.r0_count && sp.r0_start <= (uint32_t)e1) {  // overlap: merge
            sp.r1_count = 0;
            sp.r0_start = 0;
            sp.r0_count = chi;
          }
        }
        if (sp.r0_count == 0 && sp.r1_count == 0) return false;
        if (sp.r0_count == 0) {
          sp.r0_start = sp.r1_start; sp.r0_count = sp.r1_count; sp.r1_count = 0;
        }
      }
    }
  }
  if (full) {
    sp.r0_start = 0;
    sp.r0_count = chi;
    sp.r1_count = 0;
  }
  return true;
}

// The apparent-area cull of the paper's early pass (step 1, Eq.
// apparent_area), opt-in (GRCA_LOSSY_AREA): true when the triangle's solid
// angle A (c - o) . n_hat / |c - o|^3, from its local vertices, is below
// eps.  Both sides squared, so it needs no back-face test first.
__device__ inline bool below_apparent_area(const float (&x)[3], const float (&y)[3],
                                           const float (&z)[3], float eps) {
  const float e1x = x[1] - x[0], e1y = y[1] - y[0], e1z = z[1] - z[0];
  const float e2x = x[2] - x[0], e2y = y[2] - y[0], e2z = z[2] - z[0];
  const float nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
  const float cx = (x[0] + x[1] + x[2]) * (1.0f / 3.0f);
  const float cy = (y[0] + y[1] + y[2]) * (1.0f / 3.0f);
  const float cz = (z[0] + z[1] + z[2]) * (1.0f / 3.0f);
  const float a = 0.5f * fmaf(cx, nx, fmaf(cy, ny, cz * nz));  // A (c - o) . n_hat
  const float c2 = fmaf(cx, cx, fmaf(cy, cy, cz * cz));
  return a * a < eps * eps * c2 * c2 * c2;
}

// Conservative candidate span of one (triangle, sensor) pair, FP32.
// Returns false when no ray of the sensor can reach the triangle.
__device__ inline bool span_of(const float (&vx)[3], const float (&vy)[3], const float (&vz)[3],
                               const DevSensor& s, uint32_t small_c, uint32_t small_r,
                               bool need_range, bool need_pole, Span& sp) {
  float x[3], y[3], z[3], r2[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float dx = vx[k] - s.o[0], dy = vy[k] - s.o[1], dz = vz[k] - s.o[2];
    x[k] = fmaf(dx, s.f[0], fmaf(dy, s.f[1], dz * s.f[2]));
    y[k] = fmaf(dx, s.r[0], fmaf(dy, s.r[1], dz * s.r[2]));
    z[k] = fmaf(dx, s.u[0], fmaf(dy, s.u[1], dz * s.u[2]));
    r2[k] = fmaf(x[k], x[k], fmaf(y[k], y[k], z[k] * z[k]));
  }
  // range, vertical noise and lossy bits in one 16-byte load
  const float4 rn = *reinterpret_cast<const float4*>(&s.dmin);
  const float dmin = rn.x, dmax = rn.y, el_noise = rn.z;
  // the opt-in lossy apparent-area cull (the same for every lane of a cast)
  if ((__float_as_uint(rn.w) & GRCA_LOSSY_AREA) && below_apparent_area(x, y, z, s.eps_area))
    return false;
  // Vertical axis through the origin vs the triangle's horizontal projection
  // (first, so that the world-space vertices and the sensor's f and r are
  // not needed past this point).
  bool pole = false;
  if (need_pole) {
    // The projection can only surround the axis if its bounding box holds
    // the origin (margin well above the FP32 error of the local coordinates).
    const float mg = 1e-6f * __builtin_amdgcn_sqrtf(fmaxf(r2[0], fmaxf(r2[1], r2[2])));
    const bool box_out = (x[0] > mg && x[1] > mg && x[2] > mg) ||
                         (x[0] < -mg && x[1] < -mg && x[2] < -mg) ||
                         (y[0] > mg && y[1] > mg && y[2] > mg) ||
                         (y[0] < -mg && y[1] < -mg && y[2] < -mg);
    if (!box_out) {
      // 2D edge functions q_k x (q_{k+1} - q_k), the edge taken from the
      // world-space vertex difference so that no cancellation sets the error
      float e[3], tol[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int k1 = (k + 1) % 3;
        const float ex = vx[k1] - vx[k], ey = vy[k1] - vy[k], ez = vz[k1] - vz[k];
        const float dxl = fmaf(ex, s.f[0], fmaf(ey, s.f[1], ez * s.f[2]));
        const float dyl = fmaf(ex, s.r[0], fmaf(ey, s.r[1], ez * s.r[2]));
        e[k] = x[k] * dyl - y[k] * dxl;
        tol[k] = 4e-6f * __builtin_amdgcn_sqrtf(r2[k]) * (fabsf(dxl) + fabsf(dyl));
      }
      const bool in_pos = e[0] >= -tol[0] && e[1] >= -tol[1] && e[2] >= -tol[2];
      const bool in_neg = e[0] <= tol[0] && e[1] <= tol[1] && e[2] <= tol[2];
      pole = in_pos || in_neg;
    }
  }
  // range prefilter: the triangle lies inside the blind ball (convex), or its
  // bounding sphere lies beyond range_max.
  if (need_range) {
    const float r2max = fmaxf(r2[0], fmaxf(r2[1], r2[2]));
    if (r2max < dmin * dmin * (1.0f - 1e-5f)) return false;
    const float cx = (x[0] + x[1] + x[2]) * (1.0f / 3.0f);
    const float cy = (y[0] + y[1] + y[2]) * (1.0f / 3.0f);
    const float cz = (z[0] + z[1] + z[2]) * (1.0f / 3.0f);
    float rc2 = 0.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float ex = x[k] - cx, ey = y[k] - cy, ez = z[k] - cz;
      rc2 = fmaxf(rc2, fmaf(ex, ex, fmaf(ey, ey, ez * ez)));
    }
    // |c| - r_c > D_max  <=>  |c|^2 > (D_max + r_c)^2 (both sides non-negative)
    const float reach = dmax * (1.0f + 1e-5f) + 1e-6f + __builtin_amdgcn_sqrtf(rc2) * 1.0001f;
    if (fmaf(cx, cx, fmaf(cy, cy, cz * cz)) > reach * reach * (1.0f + 1e-5f)) return false;
  }
  const float r2min = fminf(r2[0], fminf(r2[1], r2[2]));
  float s_lo, s_hi;
  bool full = false;
  if (!(r2min > 1e-24f)) {
    // a vertex (numerically) at the origin: no usable extent, take everything
    s_lo = -1.0f; s_hi = 1.0f; full = true;
  } else {
    // r2 >= 1e-24 is a normal float: the hardware reciprocal square root
    // (1 ulp) needs no denormal scaling
    float inv[3], sn[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      inv[k] = __builtin_amdgcn_rsqf(r2[k]);
      sn[k] = z[k] * inv[k];
    }
    s_lo = fminf(sn[0], fminf(sn[1], sn[2]));
    s_hi = fmaxf(sn[0], fmaxf(sn[1], sn[2]));
    // Edge bulge: along a great-circle arc of angle L between unit endpoints
    // a, b every point is c/|c| with c on the chord and |c| >= cos(L/2), so
    // the arc's sine-elevation stays within [min(m, m/cos), max(M, M/cos)].
    float cmin = 1.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int k1 = (k + 1) % 3;
      const float c = fmaf(x[k], x[k1], fmaf(y[k], y[k1], z[k] * z[k1])) * inv[k] * inv[k1];
      cmin = fminf(cmin, c);
    }
    const float kb = __builtin_amdgcn_rsqf(fmaxf(0.5f * (1.0f + cmin), 1e-12f)) * (1.0f + 1e-6f);
    if (s_hi > 0.0f) s_hi = fminf(s_hi * kb, 1.0f);
    if (s_lo < 0.0f) s_lo = fmaxf(s_lo * kb, -1.0f);
    // the projection surrounds the vertical axis: every elevation on the
    // side(s) of the horizon the triangle reaches
    if (pole) {
      full = true;
      const bool up = z[0] > 0.0f && z[1] > 0.0f && z[2] > 0.0f;
      const bool dn = z[0] < 0.0f && z[1] < 0.0f && z[2] < 0.0f;
      if (!dn) s_hi = 1.0f;
      if (!up) s_lo = -1.0f;
    }
  }
  const float smax_abs = fmaxf(fabsf(s_lo), fabsf(s_hi));
  // (vertical noise: |sin(phi + o) - sin(phi)| <= |o|)
  s_lo -= ETA_SIN + el_noise;
  s_hi += ETA_SIN + el_noise;
  // both bin loads in flight together
  const ChanBin e_lo = load_bin(s.bins + chan_bin(s, s_lo));
  const ChanBin e_hi = load_bin(s.bins + chan_bin(s, s_hi));
  const uint32_t c_from = chan_resolve(s, e_lo, s_lo, false);
  const uint32_t c_end = chan_resolve(s, e_hi, s_hi, true);
  if (c_from >= c_end) return false;
  sp.c_from = c_from;
  sp.c_count = c_end - c_from;
  if (smax_abs > S_POLE) full = true;

  if (!ray_span(x, y, smax_abs, full, s, sp)) return false;
  sp.large = full || sp.c_count > small_c || sp.r0_count > small_r ||
             (sp.r1_count > small_r);
  return true;
}

// ------------------------------------------------------------ lossy modes
// The paper's own early pass, opt-in (GRCA_LOSSY_* cast flags): FP32 with
// no margins, so rays near a triangle's angular boundary can lose their hit
// (its accuracy section lists these as causes 1, 2 and 3).

// GACP-T boolean predicate (section 3.5, "Boolean predicate"): does the cone
// of elevation phi (sine sphi) around the up axis through the origin cross
// the triangle?  Local coordinates (z up), |p_k| given as inv[k] = 1 / |p_k|.
// Vertex classification first: all below the origin's horizontal plane (for
// phi > 0; above, for phi < 0) -> no; all inside the cone -> no; some inside
// and some outside -> yes; all outside -> the apex-ray check (the axis ray
// of the cone's side hits the triangle, and the triangle lies within
// range_max |sin phi| of the origin; its plane distance stands in for the
// closest-point distance), then the per-edge quadratic
//   (e_A^2 - s^2 |e|^2) l^2 + 2 (e_A h - s^2 p.e) l + (h^2 - s^2 |p|^2) = 0
// with a root l in [0, 1] on the cone's forward half.  phi = 0 is the plane
// case: the heights change sign.
__device__ inline bool gacp_t(const float (&x)[3], const float (&y)[3], const float (&z)[3],
                              const float (&inv)[3], float sphi, bool apex_up, bool apex_dn,
                              float plane_dist, float dmax) {
  if (sphi == 0.0f) {
    const bool pos = z[0] > 0.0f || z[1] > 0.0f || z[2] > 0.0f;
    const bool neg = z[0] < 0.0f || z[1] < 0.0f || z[2] < 0.0f;
    return (pos && neg) || z[0] == 0.0f || z[1] == 0.0f || z[2] == 0.0f;
  }
  const float sg = sphi > 0.0f ? 1.0f : -1.0f;
  const float sa = fabsf(sphi);
  float h[3];
  int inside = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    h[k] = sg * z[k];
    inside += (h[k] * inv[k] >= sa) ? 1 : 0;
  }
  if (h[0] < 0.0f && h[1] < 0.0f && h[2] < 0.0f) return false;  // wrong half-space
  if (inside == 3) return false;
  if (inside > 0) return true;
  if ((sg > 0.0f ? apex_up : apex_dn) && plane_dist <= dmax * sa) return true;
  const float s2 = sa * sa;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int k1 = (k + 1) % 3;
    const float ex = x[k1] - x[k], ey = y[k1] - y[k], ez = z[k1] - z[k];
    const float ea = sg * ez;
    const float pe = fmaf(x[k], ex, fmaf(y[k], ey, z[k] * ez));
    const float ee = fmaf(ex, ex, fmaf(ey, ey, ez * ez));
    const float pp = fmaf(x[k], x[k], fmaf(y[k], y[k], z[k] * z[k]));
    const float c2 = fmaf(ea, ea, -s2 * ee);
    const float c1 = 2.0f * fmaf(ea, h[k], -s2 * pe);
    const float c0 = fmaf(h[k], h[k], -s2 * pp);
    const float disc = fmaf(c1, c1, -4.0f * c2 * c0);
    if (disc < 0.0f) continue;
    float l0, l1;
    if (c2 == 0.0f) {
      if (c1 == 0.0f) continue;
      l0 = l1 = -c0 / c1;
    } else {
      const float sq = sqrtf(disc);
      l0 = (-c1 - sq) / (2.0f * c2);
      l1 = (-c1 + sq) / (2.0f * c2);
    }
    if (l0 >= 0.0f && l0 <= 1.0f && fmaf(l0, ea, h[k]) >= 0.0f) return true;
    if (l1 >= 0.0f && l1 <= 1.0f && fmaf(l1, ea, h[k]) >= 0.0f) return true;
  }
  return false;
}

// span_of with the paper's lossy steps enabled by s.lossy:
//  GRCA_LOSSY_AREA   cull when the apparent area A (c - o) . n / |c - o|^3
//                    (early pass step 1) is below eps_area;
//  GRCA_LOSSY_CSPAN  the channel span by two binary searches with gacp_t,
//                    both started at C_mid, the channel midway between the
//                    vertices' nearest channels on the uniform grid (section
//                    3.6); no crossing at C_mid discards the pair;
//  GRCA_LOSSY_RSPAN  when all three vertices lie on one side of the sensor
//                    (all-front along the centre ray, all-right or all-left,
//                    Eq. all_cw; always for fields of view up to 180
//                    degrees), the ray span from the vertex azimuths rounded
//                    to the nearest ray and clamped to the sensor (section
//                    3.7); otherwise the pair takes the large class, whose
//                    per-channel arcs are exact.
// Steps not enabled are the exact ones of span_of.
__device__ inline bool span_of_lossy(const float (&vx)[3], const float (&vy)[3],
                                     const float (&vz)[3], const DevSensor& s, uint32_t small_c,
                                     uint32_t small_r, bool need_range, bool need_pole,
                                     Span& sp) {
  const uint32_t lossy = s.lossy;
  float x[3], y[3], z[3], r2[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float dx = vx[k] - s.o[0], dy = vy[k] - s.o[1], dz = vz[k] - s.o[2];
    x[k] = fmaf(dx, s.f[0], fmaf(dy, s.f[1], dz * s.f[2]));
    y[k] = fmaf(dx, s.r[0], fmaf(dy, s.r[1], dz * s.r[2]));
    z[k] = fmaf(dx, s.u[0], fmaf(dy, s.u[1], dz * s.u[2]));
    r2[k] = fmaf(x[k], x[k], fmaf(y[k], y[k], z[k] * z[k]));
  }
  if ((lossy & GRCA_LOSSY_AREA) && below_apparent_area(x, y, z, s.eps_area)) return false;
  // face normal n = e1 x e2 (|n| = 2 A), local axes
  const float e1x = x[1] - x[0], e1y = y[1] - y[0], e1z = z[1] - z[0];
  const float e2x = x[2] - x[0], e2y = y[2] - y[0], e2z = z[2] - z[0];
  const float nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
  // the up axis through the origin against the triangle's horizontal projection
  bool pierce = false;
  {
    float e[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int k1 = (k + 1) % 3;
      e[k] = x[k] * (y[k1] - y[k]) - y[k] * (x[k1] - x[k]);
    }
    pierce = (e[0] >= 0.0f && e[1] >= 0.0f && e[2] >= 0.0f) ||
             (e[0] <= 0.0f && e[1] <= 0.0f && e[2] <= 0.0f);
  }
  bool pole = false;
  if (need_pole) pole = pierce;
  const float dmin = s.dmin, dmax = s.dmax;
  if (need_range) {
    const float r2max = fmaxf(r2[0], fmaxf(r2[1], r2[2]));
    if (r2max < dmin * dmin) return false;
    const float r2min = fminf(r2[0], fminf(r2[1], r2[2]));
    // plane distance as the closest-point distance: beyond range_max
    const float nn = fmaf(nx, nx, fmaf(ny, ny, nz * nz));
    const float g = fmaf(x[0], nx, fmaf(y[0], ny, z[0] * nz));
    if (nn > 0.0f && g * g > dmax * dmax * nn && r2min > dmax * dmax) return false;
  }
  const float r2min = fminf(r2[0], fminf(r2[1], r2[2]));
  if (!(r2min > 1e-24f)) return span_of(vx, vy, vz, s, small_c, small_r, need_range, need_pole, sp);
  float inv[3], sn[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    inv[k] = __builtin_amdgcn_rsqf(r2[k]);
    sn[k] = z[k] * inv[k];
  }
  const uint32_t gamma = s.gamma;
  uint32_t c_from, c_end;
  bool full = false;
  // largest |sine of elevation| (the azimuth margin near the poles)
  float smax_abs = fmaxf(fabsf(sn[0]), fmaxf(fabsf(sn[1]), fabsf(sn[2])));
  if (lossy & GRCA_LOSSY_CSPAN) {
    // apex ray: the up (down) axis meets the triangle's plane above (below)
    // the origin inside the triangle
    const float g = fmaf(x[0], nx, fmaf(y[0], ny, z[0] * nz));  // n . p0
    const bool up = pierce && nz != 0.0f && g / nz > 0.0f;
    const bool dn = pierce && nz != 0.0f && g / nz < 0.0f;
    const float nn = fmaf(nx, nx, fmaf(ny, ny, nz * nz));
    const float plane_dist = nn > 0.0f ? fabsf(g) * __builtin_amdgcn_rsqf(nn) : 0.0f;
    int cmin = (int)gamma, cmax = -1;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float ci = rintf((asinf(fminf(fmaxf(sn[k], -1.0f), 1.0f)) - s.elev0) * s.inv_delev);
      const int c = (int)fminf(fmaxf(ci, 0.0f), (float)(gamma - 1u));
      cmin = min(cmin, c);
      cmax = max(cmax, c);
    }
    const int cmid = (cmin + cmax + 1) / 2;
    auto crosses = [&](int j) {
      return gacp_t(x, y, z, inv, s.sin_tab[j], up, dn, plane_dist, dmax);
    };
    if (!crosses(cmid)) return false;
    int lo = 0, hi = cmid;
    while (lo < hi) {
      const int m = (lo + hi) / 2;
      if (crosses(m)) hi = m; else lo = m + 1;
    }
    c_from = (uint32_t)lo;
    lo = cmid;
    hi = (int)gamma - 1;
    while (lo < hi) {
      const int m = (lo + hi + 1) / 2;
      if (crosses(m)) lo = m; else hi = m - 1;
    }
    c_end = (uint32_t)lo + 1u;
    if (pole) full = true;
  } else {
    // the exact elevation extent of span_of
    float s_lo = fminf(sn[0], fminf(sn[1], sn[2]));
    float s_hi = fmaxf(sn[0], fmaxf(sn[1], sn[2]));
    float cmn = 1.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int k1 = (k + 1) % 3;
      cmn = fminf(cmn, fmaf(x[k], x[k1], fmaf(y[k], y[k1], z[k] * z[k1])) * inv[k] * inv[k1]);
    }
    const float kb = __builtin_amdgcn_rsqf(fmaxf(0.5f * (1.0f + cmn), 1e-12f)) * (1.0f + 1e-6f);
    if (s_hi > 0.0f) s_hi = fminf(s_hi * kb, 1.0f);
    if (s_lo < 0.0f) s_lo = fmaxf(s_lo * kb, -1.0f);
    if (pole) {
      full = true;
      const bool up = z[0] > 0.0f && z[1] > 0.0f && z[2] > 0.0f;
      const bool dn = z[0] < 0.0f && z[1] < 0.0f && z[2] < 0.0f;
      if (!dn) s_hi = 1.0f;
      if (!up) s_lo = -1.0f;
    }
    smax_abs = fmaxf(fabsf(s_lo), fabsf(s_hi));
    if (smax_abs > S_POLE) full = true;
    s_lo -= ETA_SIN + s.el_noise;
    s_hi += ETA_SIN + s.el_noise;
    c_from = chan_search(s, s_lo, false);
    c_end = chan_search(s, s_hi, true);
  }
  if (c_from >= c_end) return false;
  sp.c_from = c_from;
  sp.c_count = c_end - c_from;
  sp.r1_start = 0;
  sp.r1_count = 0;
  const uint32_t chi = s.chi;
  if (!full && (lossy & GRCA_LOSSY_RSPAN)) {
    bool all_cw = !s.wrap && (float)chi <= s.period_idx * 0.5f;  // field of view <= 180 deg
    if (!all_cw) {
      // centre ray (channel floor(gamma / 2), azimuth 0) and a right vector
      // by Gram-Schmidt from the up axis (the forward axis near the poles)
      const float2 cc = s.chan[gamma / 2u];
      const float dx = cc.x, dz = cc.y;  // (cos phi_c, 0, sin phi_c)
      const bool steep = fabsf(dz) >= 0.9f;
      const float wx = steep ? 1.0f : 0.0f, wz = steep ? 0.0f : 1.0f;
      const float wd = wx * dx + wz * dz;
      float ux = wx - wd * dx, uz = wz - wd * dz;
      const float iu = __builtin_amdgcn_rsqf(fmaf(ux, ux, uz * uz));
      ux *= iu;
      uz *= iu;
      // r_perp = d x u_perp, d and u_perp in the x-z plane: (0, dz ux - dx uz, 0)
      const float ry = dz * ux - dx * uz;
      bool front = true, right = true, left = true;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        front = front && fmaf(x[k], dx, z[k] * dz) > 0.0f;
        right = right && y[k] * ry > 0.0f;
        left = left && y[k] * ry < 0.0f;
      }
      all_cw = front || right || left;
    }
    if (all_cw) {
      int rmin = (int)chi, rmax = -1;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float t = atan2f(y[k], x[k]);
        const float ri = rintf((t - s.theta_start) * s.inv_dtheta);
        const int r = (int)fminf(fmaxf(ri, 0.0f), (float)(chi - 1u));
        rmin = min(rmin, r);
        rmax = max(rmax, r);
      }
      sp.r0_start = (uint32_t)rmin;
      sp.r0_count = (uint32_t)(rmax - rmin + 1);
    } else {
      full = true;  // the seam case: large class
    }
    if (full) {
      sp.r0_start = 0;
      sp.r0_count = chi;
    }
    sp.large = full || sp.c_count > small_c || sp.r0_count > small_r;
    return true;
  }
  // the exact azimuth arc of span_of
  if (smax_abs > S_POLE) full = true;
  if (!ray_span(x, y, smax_abs, full, s, sp)) return false;
  sp.large = full || sp.c_count > small_c || sp.r0_count > small_r || sp.r1_count > small_r;
  return true;
}

// Sphere culling (the "group" extension of the cone-triangle test): a group
// of triangles, a 128-triangle bounds tile or a single triangle, is bounded
// by a sphere (centre c, radius rad).  The verdict is `culled` when no ray of
// sensor `s` can reach anything inside the sphere: it lies beyond range_max,
// or the band of elevations it subtends holds no channel, or (AZ, on a
// partial-FOV sensor) the azimuths it subtends miss the field of view.
// Conservative: any doubt (sphere near the origin, wide angles) keeps it.
struct GroupVerdict {
  bool culled;      // no ray of the sensor can reach the group
  bool need_range;  // the group straddles range_min or range_max: test triangles
  bool need_pole;   // the group touches the vertical axis through the origin
  bool need_fov;    // (AZ) the group straddles the edge of a partial field of view
};

// A sphere (centre at local lf, lr; distance D from the origin; radius r
// widened) against the wedge of a partial field of view: `out` when it lies
// wholly outside (no ray of the sensor can reach it), `in` when wholly
// inside.  The signed distance of the centre from each bounding plane is one
// dot product with the plane's inward normal, and every point of the sphere
// lies within r of it.  The margin 1e-5 D covers the FP32 error of the local
// frame and of the rounded normals (under 1e-6 D); the widening of the wedge
// by 1e-4 rad covers the rounded ray directions.  NaN (D = 0) gives neither.
struct FovVerdict {
  bool out, in;
};
__device__ inline FovVerdict fov_verdict(float lf, float lr, float D, float r,
                                         const DevSensor& s) {
  const float a1 = fmaf(s.fov_n[0], lf, s.fov_n[1] * lr);
  const float a2 = fmaf(s.fov_n[2], lf, s.fov_n[3] * lr);
  const float rp = fmaf(1e-5f, D, r + 1e-6f);
  const bool o1 = a1 < -rp, o2 = a2 < -rp, i1 = a1 > rp, i2 = a2 > rp;
  const bool convex = s.fov_mode == 1u;
  FovVerdict v;
  v.out = s.fov_mode != 0u && (convex ? (o1 || o2) : (o1 && o2));
  v.in = s.fov_mode == 0u || (convex ? (i1 && i2) : (i1 || i2));
  return v;
}

// A non-negative float as the bits of the next FP16 value at or above it
// (+inf above the FP16 range), and back.
__device__ inline uint32_t half_up(float x) {
  const _Float16 h = (_Float16)x;
  uint32_t b = (uint32_t)__builtin_bit_cast(uint16_t, h);
  if ((float)h < x) ++b;
  return b;
}
__device__ inline float unpack_half(uint32_t b) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)b);
}

// The bounds of a triangle or a tile (centre c; an upright cylinder about c
// packed in `rad`, and the sphere about c that holds the cylinder) against
// sensor `s`, without memory access besides the sensor's fields (read
// together); about 80 FP32 operations, 90 with AZ.
// Culled when the sphere lies beyond range_max, when no channel elevation
// lies within alpha of the elevation of c, or (AZ, partial field of view)
// when it lies outside the field of view's wedge.  For
// sin(alpha) = r / D <= 1/2 every point of the sphere is within the angle
// alpha <= asin(r / D) <= (r / D)(1 + (r / D)^2 / 3) of c's direction, so its
// elevation is within alpha of c's.  The channels are taken as the uniform grid elev0 + j / inv_delev,
// widened by elev_tol (the table's largest distance from that grid); the
// margins cover the FP32 error of c's angles and of the ray test.
// need_range: the sphere straddles range_min or range_max; need_pole: it
// touches the vertical axis through the origin.  Used for bounds tiles (AZ)
// and for single triangles.  want_range / want_pole / want_fov (wave-uniform)
// skip the parts whose verdict the caller will not use: false gives
// need_range = need_pole = false and no field-of-view test.
//
// `rad` holds the bits of a packed cylinder (pack_cylinder) of the triangle
// or tile: horizontal radius rh and vertical half-height hz about c,
// both already widened.  The sphere radius is then sqrt(rh^2 + hz^2), and for
// a sensor whose up axis is the world z axis the angular margin is the
// cylinder's instead of the sphere's: every point of the triangle has height
// z within hz of c's and horizontal distance rho within rh of c's, and on that
// box in the (z, rho) plane the elevation atan2(z, rho) has
// |d/dz| = rho / D^2 <= (rho_c + rh) / D_min^2 and |d/drho| = |z| / D^2 <=
// (|z_c| + hz) / D_min^2, with D_min >= D - r, so that (mean value theorem)
// its elevation is within ((rho_c + rh) hz + (|z_c| + hz) rh) / (D - r)^2 of
// c's.  For a ground triangle at a shallow angle (hz ~ 0) that is sin|el|
// times the sphere's margin.
template <bool AZ>
__device__ inline GroupVerdict sphere_test(float cx, float cy, float cz, float rad,
                                           const DevSensor& s, bool want_range = true,
                                           bool want_pole = true, bool want_fov = true) {
  float r, rh, hz;
  {
    uint32_t pk = __float_as_uint(rad);
    // (an empty asm that the compiler must take as changing pk: the unpacked
    // values are recomputed per test rather than hoisted out of the caller's
    // sensor loop, where they would hold three more registers per triangle)
    asm volatile("" : "+v"(pk));
    rh = unpack_half(pk & 0xFFFFu);
    hz = unpack_half(pk >> 16);
    r = __builtin_amdgcn_sqrtf(fmaf(rh, rh, hz * hz));
  }
  const float dx = cx - s.o[0], dy = cy - s.o[1], dz = cz - s.o[2];
  const float lf = fmaf(dx, s.f[0], fmaf(dy, s.f[1], dz * s.f[2]));
  const float lr = fmaf(dx, s.r[0], fmaf(dy, s.r[1], dz * s.r[2]));
  const float lu = fmaf(dx, s.u[0], fmaf(dy, s.u[1], dz * s.u[2]));
  const float h2 = fmaf(lf, lf, lr * lr);
  const float D2 = fmaf(lu, lu, h2);
  const float r2 = r * r;
  const bool near = D2 <= 4.0f * r2;  // the origin is within 2r: keep
  const float invD = __builtin_amdgcn_rsqf(D2);
  const float D = D2 * invD;
  const bool beyond = D - r > s.cull_dmax;
  // elevation of c (in [-pi/2, pi/2], |error| <= 2e-6; NaN only at D = 0,
  // where the sphere is near)
  const float hc = __builtin_amdgcn_sqrtf(h2);
  float m;
  if (s.upright) {
    // (used only when far: D > 2 r, so D - r > r > 0; the factor 1.0001
    // covers the FP32 error of D - r)
    const float inv = __builtin_amdgcn_rcpf(D - r);
    const float num = fmaf(hc + rh, hz, (fabsf(lu) + hz) * rh);
    m = fmaf(num * inv, inv * 1.0001f, s.elev_m);
  } else {
    const float sa = r * invD;
    m = fmaf(sa * sa * (1.0f / 3.0f), sa, sa) + s.elev_m;
  }
  const float el = atan2_right(lu, hc);
  // grid coordinates of el -+ m: (el - elev0) / delev -+ m / delev (the
  // roundings are a few ulps of a channel index, far inside the margin)
  const float eg = fmaf(el, s.inv_delev, -s.elev0_g);
  const float mg = m * s.inv_delev;
  const float j_lo = ceilf(eg - mg);
  const float j_hi = floorf(eg + mg);
  // some channel index j in [max(j_lo, 0), min(j_hi, gamma - 1)]; written
  // with negated comparisons, so that a NaN keeps the sphere
  const bool band = (uint32_t)!(j_lo > j_hi) & (uint32_t)!(j_lo > s.last_chan) &
                    (uint32_t)!(j_hi < 0.0f);
  uint32_t out_fov = 0u, in_fov = 1u;
  if (AZ && want_fov) {
    const FovVerdict fv = fov_verdict(lf, lr, D, r, s);
    out_fov = (uint32_t)fv.out;
    in_fov = (uint32_t)fv.in;
  }
  // (bitwise: a short-circuit would add branches)
  const uint32_t far = (uint32_t)!near;
  GroupVerdict v;
  v.culled = (far & ((uint32_t)beyond | (uint32_t)!band | out_fov)) != 0u;
  v.need_range = false;
  if (want_range) {
    const bool inside = (uint32_t)(D + r < s.in_dmax) & (uint32_t)(D - r > s.in_dmin);
    v.need_range = ((uint32_t)near | (uint32_t)!inside) != 0u;
  }
  v.need_pole = want_pole && !(h2 > r2 * 1.0001f);
  v.need_fov = in_fov == 0u;
  return v;
}

// Wave-wide minimum / maximum of floats by DPP row shifts and broadcasts (no
// LDS round trips), read from the last lane: a wave-uniform value.  The
// reduction is a maximum of unsigned keys with the order of the floats (the
// complement for a minimum), for which 0, what a lane whose DPP source is
// absent reads, is neutral; no NaN quieting is needed either.
__device__ inline uint32_t float_ukey(float x) {
  const uint32_t b = __float_as_uint(x);
  return b ^ ((uint32_t)((int)b >> 31) | 0x80000000u);
}
__device__ inline float ukey_float(uint32_t k) {
  return __uint_as_float(k ^ (((k >> 31) - 1u) | 0x80000000u));
}
__device__ inline uint32_t wave_max_key(uint32_t v) {
#define GRCA_DPP_STEP(CTRL, ROWS) \
  v = max(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, ROWS, 0xf, true));
  GRCA_DPP_STEP(0x111, 0xf)  // row_shr:1
  GRCA_DPP_STEP(0x112, 0xf)  // row_shr:2
  GRCA_DPP_STEP(0x114, 0xf)  // row_shr:4
  GRCA_DPP_STEP(0x118, 0xf)  // row_shr:8
  GRCA_DPP_STEP(0x142, 0xa)  // row_bcast:15
  GRCA_DPP_STEP(0x143, 0xc)  // row_bcast:31
#undef GRCA_DPP_STEP
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}
__device__ inline float wave_max_dpp(float x) { return ukey_float(wave_max_key(float_ukey(x))); }
// Wave-wide sum by the same DPP steps (0, what an absent source reads, is
// neutral), read from the last lane.
__device__ inline float wave_sum_dpp(float x) {
#define GRCA_DPP_ADD(CTRL, ROWS) \
  x += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, ROWS, 0xf, true));
  GRCA_DPP_ADD(0x111, 0xf)  // row_shr:1
  GRCA_DPP_ADD(0x112, 0xf)  // row_shr:2
  GRCA_DPP_ADD(0x114, 0xf)  // row_shr:4
  GRCA_DPP_ADD(0x118, 0xf)  // row_shr:8
  GRCA_DPP_ADD(0x142, 0xa)  // row_bcast:15
  GRCA_DPP_ADD(0x143, 0xc)  // row_bcast:31
#undef GRCA_DPP_ADD
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}
__device__ inline float wave_min_dpp(float x) { return ukey_float(~wave_max_key(~float_ukey(x))); }

// Block b's place in tile order.  Blocks are handed to the 8 XCDs round
// robin and each XCD takes its blocks in order; here every XCD gets runs of
// `run` consecutive blocks (neighbouring triangles share vertices in the
// XCD's L2), the runs dealt to the XCDs in turn, so that all XCDs move
// through the scene together and finish together whatever the distribution
// of work in it.  Longer runs fetch fewer vertex lines twice (from two
// XCDs); runs of 256 tiles cost no time over 64.  Blocks past the last full
// round of runs keep their index.
constexpr uint32_t XCD_RUN_TILES = 256;
__device__ inline uint32_t xcd_chunked(uint32_t b, uint32_t nb, uint32_t run) {
  const uint32_t full = nb / (8u * run) * (8u * run);
  if (b >= full) return b;
  const uint32_t x = b % 8u, k = b / 8u;
  return ((k / run) * 8u + x) * run + k % run;
}

// Candidate pairs of a work item (rectangle or row).
__device__ inline uint32_t item_candidates(const Item& it) {
  return (it.chan >> 16) * (it.rays >> 16);
}

// Bounds pass, one 128-triangle tile per wave: lane l holds triangles l
// and 64 + l of the tile, so that every memory round trip of the wave serves
// two triangles.  Two phases over the sensors observing the tile's scene:
//  1. one bounding-sphere test of the whole tile (lane k tests sensor k of
//     each run of 64 sensors) skips a sensor; otherwise each lane tests its
//     triangles' own bounding spheres against the sensor (elevation band,
//     range, and the field of view where the tile straddles its edge) and
//     the surviving (triangle, sensor) pairs are queued in the wave's LDS
//     ring;
//  2. whenever 64 pairs are queued, and at the end, every lane takes one
//     pair, reads the triangle's vertices (from LDS, or from the record
//     copies for a tile of static triangles) and computes the pair's
//     candidate span, with the sensor read per lane.
// Most pairs that pass the tile's test fail their triangle's own test (small
// triangles between two channels), so the span, the costly part, runs on
// full waves of likely survivors rather than on every lane of every sensor.
// The records of a span batch go to the tile's item shard (small class) and
// large-record shard (large class) with one atomic each.
// Resident waves per SIMD the plain bounds pass is compiled for: 7 leaves it
// 72 VGPRs, enough for the span phase without spills (at 8 waves, 64 VGPRs,
// the spills cost more than the extra wave gains).
constexpr int BOUNDS_WAVES_PER_SIMD = 7;

// Bounding cylinders of a lane's two triangles (about the AABB centre) and
// of the wave's 128-triangle tile (wave-uniform: about the mean of the 128
// slots' triangle centres; any centre will do, and a slot past the scene's
// end holds a copy of the tile's first triangle, so no masks).  The same
// arithmetic at scene setup and in the bounds pass.
// A cylinder about a centre, widened and packed into one word: horizontal radius rh (low half) and vertical half-height hz (high
// half), each widened by 1e-4 relative, 2e-4 of the other (a sensor up axis
// up to 1e-4 off the z axis mixes the two) and 1e-6 m, rounded up to FP16.
__device__ inline uint32_t pack_cylinder(float rh, float hz) {
  const float a = fmaf(rh, 1.0001f, fmaf(hz, 2e-4f, 1e-6f));
  const float b = fmaf(hz, 1.0001f, fmaf(rh, 2e-4f, 1e-6f));
  return half_up(a) | (half_up(b) << 16);
}

// Each of a lane's two triangles: AABB centre in tc[h][0..2], the bits of
// its packed cylinder in tc[h][3].
__device__ inline void tri_spheres(const float (&v)[2][9], float (&tc)[2][4]) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    float mn[3], mx[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      mn[c] = fminf(v[h][c], fminf(v[h][3 + c], v[h][6 + c]));
      mx[c] = fmaxf(v[h][c], fmaxf(v[h][3 + c], v[h][6 + c]));
      tc[h][c] = 0.5f * (mn[c] + mx[c]);
    }
    float rh2 = 0.0f, hz = 0.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float ex = v[h][3 * k] - tc[h][0], ey = v[h][3 * k + 1] - tc[h][1],
                  ez = v[h][3 * k + 2] - tc[h][2];
      rh2 = fmaxf(rh2, fmaf(ex, ex, ey * ey));
      hz = fmaxf(hz, fabsf(ez));
    }
    // hardware square root (1 ulp; a denormal rh2 may give 0): covered by
    // the widening
    tc[h][3] = __uint_as_float(pack_cylinder(__builtin_amdgcn_sqrtf(rh2), hz));
  }
}
__device__ inline void tile_sphere(const float (&v)[2][9], const float (&tc)[2][4],
                                   float (&gs)[4]) {
  float g[3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
    g[c] = first_lane(wave_sum_dpp(tc[0][c] + tc[1][c]) * (1.0f / 128.0f));
  float rh2 = 0.0f, hz = 0.0f;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float ex = v[h][3 * k] - g[0], ey = v[h][3 * k + 1] - g[1],
                  ez = v[h][3 * k + 2] - g[2];
      rh2 = fmaxf(rh2, fmaf(ex, ex, ey * ey));
      hz = fmaxf(hz, fabsf(ez));
    }
  }
  gs[0] = g[0];
  gs[1] = g[1];
  gs[2] = g[2];
  gs[3] = __uint_as_float(first_lane(
      pack_cylinder(__builtin_amdgcn_sqrtf(wave_max_dpp(rh2)), wave_max_dpp(hz))));
}

// Scene setup: the spheres of the n_pre leading tiles, one wave per tile,
// from the static triangles' vertex records.
__global__ __launch_bounds__(256) void sphere_kernel(const float4* __restrict__ soup,
                                                     uint32_t n_pre, float4* __restrict__ tsph,
                                                     float4* __restrict__ gsph) {
  const uint32_t tile = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (tile >= n_pre) return;  // wave-uniform
  const uint32_t lane = lane_id();
  float v[2][9];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const uint32_t t = tile * BOUNDS_TILE + 64u * h + lane;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float4 p = soup[3ull * t + k];
      v[h][3 * k] = p.x;
      v[h][3 * k + 1] = p.y;
      v[h][3 * k + 2] = p.z;
    }
  }
  float tc[2][4], gs[4];
  tri_spheres(v, tc);
  tile_sphere(v, tc, gs);
#pragma unroll
  for (int h = 0; h < 2; ++h)
    tsph[(size_t)tile * BOUNDS_TILE + 64u * h + lane] = make_float4(tc[h][0], tc[h][1], tc[h][2], tc[h][3]);
  if (lane == 0) gsph[tile] = make_float4(gs[0], gs[1], gs[2], gs[3]);
}

template <int WPB, bool INLINE, bool LOSSY>
__global__ __launch_bounds__(WPB * 64, INLINE || LOSSY ? 1 : BOUNDS_WAVES_PER_SIMD) void bounds_kernel(
    const DevScene* __restrict__ scenes, uint32_t nscenes, uint32_t total_tiles,
    const DevSensor* __restrict__ sens, uint32_t small_c, uint32_t small_r,
    Item* __restrict__ items, uint32_t* __restrict__ item_cs, uint32_t item_scap,
    Item* __restrict__ large, uint32_t large_scap, Counters* __restrict__ cnt,
    uint32_t group_cull, uint32_t inline_max, unsigned long long* __restrict__ keys) {
  // queued pairs: a sensor step queues at most 128 and runs only while
  // fewer than 64 wait, so at most 191 are held
  constexpr uint32_t RING = 256;
  // ring entry: triangle (0..127) | need_range << 7 | need_pole << 8 | sensor << 9
  __shared__ uint32_t s_ring[WPB][RING];
  __shared__ float s_vtx[WPB][9][BOUNDS_TILE];  // the tile's vertices (x0 y0 z0 x1 .. z2), by triangle
  const uint32_t w = wave_id();
  const uint32_t lane = lane_id();
  uint32_t* const ring = s_ring[w];
  float (*const vtx)[BOUNDS_TILE] = s_vtx[w];
  const uint32_t tile = xcd_chunked(blockIdx.x, gridDim.x, XCD_RUN_TILES / WPB) * WPB + w;
  if (tile >= total_tiles) return;  // wave-uniform
  // statistics go to the tile's shard; records go to a shard that moves on
  // by one with every span batch, from the tile's: a tile near a sensor can
  // hold hundreds of times the candidates of a far one, and its batches are
  // spread over all shards instead of loading one
  const uint32_t shard = tile % NSHARD;
  uint32_t out_shard = shard;

  uint32_t sc = 0;
  while (sc + 1 < nscenes && tile >= scenes[sc + 1].tile_start) ++sc;
  const DevScene& S = scenes[sc];
  // the scene's fields as wave-uniform values: the loop below branches on them
  const uint32_t s_begin = first_lane(S.sensor_begin), s_end = first_lane(S.sensor_end);
  const uint32_t tri0 = first_lane((tile - S.tile_start) * BOUNDS_TILE);
  const uint32_t ntri = first_lane(S.ntri);
  // the lane's two triangles; lanes past the scene's last triangle load the
  // tile's first one (no branch) and are masked.  Loads take the arrays'
  // scalar bases and 32-bit byte offsets (the library keeps every scene
  // under 2^28 triangles and 2^28 vertices).  A leading all-static tile
  // reads its spheres as computed at scene setup, and the span phase reads
  // its vertices from the record copies; other tiles gather their vertices,
  // park them in LDS for the span phase and compute the spheres here.
  const bool pre = first_lane(tile - S.tile_start) < first_lane(S.n_pre);
  bool active[2];
  float tc[2][4];  // centre x, y, z and radius, per triangle
  float gs[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  if (pre) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      active[h] = true;
      const float4 q = gload_v(S.tsph, 16u * (tri0 + 64u * h + lane));
      tc[h][0] = q.x; tc[h][1] = q.y; tc[h][2] = q.z; tc[h][3] = q.w;
    }
    if (group_cull) {
      typedef float v4f __attribute__((ext_vector_type(4)));
      typedef const v4f __attribute__((address_space(4))) CT4;
      const v4f g = *(CT4*)(S.gsph + (tile - S.tile_start));
      gs[0] = first_lane(g.x); gs[1] = first_lane(g.y);
      gs[2] = first_lane(g.z); gs[3] = first_lane(g.w);
    }
  } else {
    float v[2][9];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t t = tri0 + 64u * h + lane;
      active[h] = t < ntri;
      const uint32_t tt = active[h] ? t : tri0;
      const Tri3 ti = gload_tri(S.idx, 12u * tt);
      const float4 p[3] = {gload_v(S.v, ti.a * 16u), gload_v(S.v, ti.b * 16u),
                           gload_v(S.v, ti.c * 16u)};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        v[h][3 * k] = p[k].x;
        v[h][3 * k + 1] = p[k].y;
        v[h][3 * k + 2] = p[k].z;
      }
#pragma unroll
      for (int c = 0; c < 9; ++c) vtx[c][64 * h + lane] = v[h][c];
    }
    tri_spheres(v, tc);
    if (group_cull) tile_sphere(v, tc, gs);
  }
  const uint32_t n_active = first_lane((uint32_t)(__popcll(__ballot(active[0])) +
                                                  __popcll(__ballot(active[1]))));
  unsigned long long rtic = 0ull;  // candidates tested inline by this lane
  unsigned long long g_cull = 0ull, g_range = ~0ull, g_pole = ~0ull, g_fov = 0ull;
  uint32_t tested = 0;     // triangle sphere tests of this wave (wave-uniform statistic)
  uint32_t evaluated = 0;  // spans computed by this wave (wave-uniform statistic)
  uint32_t head = 0, tail = 0;  // pairs taken from / queued into the ring
  uint32_t n = s_begin;
  for (;;) {
    if (n < s_end && tail - head < 64u) {
      // ---- phase 1: sensor n
      const uint32_t ln = (n - s_begin) & 63u;
      if (ln == 0) {
        // the tile's verdicts for the next 64 sensors in one pass: lane k
        // tests sensor n + k
        const uint32_t ns = n + lane;
        bool cul = false, nr = true, np = true, nf = false;
        if (group_cull && ns < s_end) {
          const GroupVerdict gv = sphere_test<true>(gs[0], gs[1], gs[2], gs[3], sens[ns]);
          cul = gv.culled;
          nr = gv.need_range;
          np = gv.need_pole;
          nf = gv.need_fov;
        }
        g_cull = first_lane(__ballot(cul));
        g_range = first_lane(__ballot(nr));
        g_pole = first_lane(__ballot(np));
        g_fov = first_lane(__ballot(nf));
      }
      if (!((g_cull >> ln) & 1ull)) {  // wave-uniform
        // both triangles of every lane (the sensor's fields are read once);
        // the range, pole and field-of-view parts only where the tile's own
        // test found the tile straddling a range limit, touching the
        // vertical axis or straddling the edge of a partial field of view
        const DevSensor& s = sens[n];
        const bool gr = (g_range >> ln) & 1ull, gp = (g_pole >> ln) & 1ull;
        const bool gf = (g_fov >> ln) & 1ull;
        const GroupVerdict v0 =
            sphere_test<true>(tc[0][0], tc[0][1], tc[0][2], tc[0][3], s, gr, gp, gf);
        const GroupVerdict v1 =
            sphere_test<true>(tc[1][0], tc[1][1], tc[1][2], tc[1][3], s, gr, gp, gf);
        tested += n_active;
        const bool keep0 = active[0] && !v0.culled;
        const bool keep1 = active[1] && !v1.culled;
        const uint32_t tag = n << 9;
        const uint32_t e0 = lane | ((uint32_t)v0.need_range << 7) |
                            ((uint32_t)v0.need_pole << 8) | tag;
        const uint32_t e1 = (64u + lane) | ((uint32_t)v1.need_range << 7) |
                            ((uint32_t)v1.need_pole << 8) | tag;
        const unsigned long long m0 = __ballot(keep0), m1 = __ballot(keep1);
        const uint32_t c0 = (uint32_t)__popcll(m0);
        if (keep0) ring[(tail + rank_in(m0)) % RING] = e0;
        if (keep1) ring[(tail + c0 + rank_in(m1)) % RING] = e1;
        tail = first_lane(tail + c0 + (uint32_t)__popcll(m1));
      }
      ++n;
    }
    // a batch runs when 64 pairs wait, or, once every sensor is tested, on
    // whatever waits (scalar control: the values are wave-uniform)
    const uint32_t avail = tail - head;
    if (avail < 64u) {
      if (n < s_end) continue;
      if (avail == 0u) break;
    }
    // ---- phase 2: spans of up to 64 queued pairs, one per lane
    const uint32_t cnt_b = avail < 64u ? avail : 64u;
    wave_sync();
    const bool live = lane < cnt_b;
    const uint32_t e = ring[(head + (live ? lane : 0u)) % RING];
    head = first_lane(head + cnt_b);
    evaluated += cnt_b;
    const uint32_t osh = out_shard;
    out_shard = (out_shard + 1u) % NSHARD;
    const uint32_t src = e & 127u;
    const uint32_t pn = live ? (e >> 9) : s_begin;
    float px[3], py[3], pz[3];
    if (pre) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float4 q = gload_v(S.soup, 48u * (tri0 + src) + 16u * (uint32_t)k);
        px[k] = q.x;
        py[k] = q.y;
        pz[k] = q.z;
      }
    } else {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        px[k] = vtx[3 * k][src];
        py[k] = vtx[3 * k + 1][src];
        pz[k] = vtx[3 * k + 2][src];
      }
    }
    const uint32_t ptri = tri0 + src;
    // (at most 4096 sensor slots per cast: a 32-bit offset)
    const DevSensor& s = *reinterpret_cast<const DevSensor*>(
        reinterpret_cast<const char*>(sens) + __umul24(pn, (uint32_t)sizeof(DevSensor)));
    Span sp;
    const bool ok = live && (LOSSY ? span_of_lossy(px, py, pz, s, small_c, small_r, (e >> 7) & 1u,
                                                   (e >> 8) & 1u, sp)
                                   : span_of(px, py, pz, s, small_c, small_r, (e >> 7) & 1u,
                                             (e >> 8) & 1u, sp));
    const uint32_t chan = ok ? (sp.c_from | (sp.c_count << 16)) : 0u;
    const bool is_large = ok && sp.large;
    bool rect0 = ok && !sp.large;
    const bool rect1 = rect0 && sp.r1_count > 0;
    // tiny single-piece rectangles: intersect right here, from the vertices
    // already in registers (the same statics and ray test as every path)
    const bool tiny = INLINE && rect0 && !rect1 && sp.c_count * sp.r0_count <= inline_max;
    if (INLINE && __ballot(tiny) != 0ull) {
      if (tiny) {
        Statics st;
        if (make_statics(px[0], py[0], pz[0], px[1], py[1], pz[1], px[2], py[2], pz[2], s, st)) {
          const uint32_t otri = S.orig[ptri];
          for (uint32_t c = 0; c < sp.c_count; ++c) {
            const uint32_t ch = sp.c_from + c;
            const float2 cp = s.chan[ch];
            for (uint32_t r = 0; r < sp.r0_count; ++r) {
              uint32_t ray = sp.r0_start + r;
              if (ray >= s.chi) ray -= s.chi;
              const uint32_t gl = ch * s.chi + ray;
              if (s.mask && !s.mask[gl]) continue;
              const float2 ca = s.az[ray];
              const unsigned long long key =
                  ray_test(st, cp.x, cp.y, ca.x, ca.y, s.dmin, s.dmax, otri);
              if (key != KEY_INIT) key_min(keys, s.key_offset + gl, key);
            }
          }
          rtic += (unsigned long long)(sp.c_count * sp.r0_count);
        }
      }
      rect0 = rect0 && !tiny;
    }
    const Item lg{ptri, chan, 0u, pn};
    wave_push(is_large, lg, large + (size_t)osh * large_scap, large_scap,
              reinterpret_cast<uint32_t*>(&cnt->large[osh].nc), &cnt->overflow, 2u, nullptr);
    // the batch's small-class records, each lane's rect0 then its rect1, all
    // appended to the wave's item shard with one 64-bit atomic that reserves
    // the slots (low word) and the candidate range (high word) together;
    // each record carries its first candidate index, so that within a shard
    // the candidate starts increase with the slot.  One scan of the lane's
    // candidate total (below 2^26 per lane, so the wave's total fits 32 bits).
    const unsigned long long m0 = __ballot(rect0), m1 = __ballot(rect1);
    const uint32_t c0 = first_lane((uint32_t)__popcll(m0));
    const uint32_t c1 = first_lane((uint32_t)__popcll(m1));
    if (c0 == 0u) continue;
    // (counts below 2^16: 24-bit multiplies)
    const uint32_t k0 = rect0 ? __umul24(sp.c_count, sp.r0_count) : 0u;
    const uint32_t k1 = rect1 ? __umul24(sp.c_count, sp.r1_count) : 0u;
    const uint32_t incl = wave_incl_scan(k0 + k1);
    const uint32_t cands = last_lane(incl);
    Shard& sh = cnt->items[osh];
    unsigned long long old = 0ull;
    if (lane == 0) {
      old = atomicAdd(&sh.nc, (unsigned long long)(c0 + c1) | ((unsigned long long)cands << 32));
      // candidate index space of the shard (2^31, so tickets cannot wrap) exhausted
      if ((uint32_t)(old >> 32) > CAND_LIMIT - cands) atomicOr(&cnt->overflow, 4u);
    }
    old = first_lane(old);
    const uint32_t base = (uint32_t)old, cbase = (uint32_t)(old >> 32);
    Item* const q_items = items + (size_t)osh * item_scap;
    uint32_t* const q_cs = item_cs + (size_t)osh * item_scap;
    // records of the lanes below (a rect1 implies the lane's rect0)
    const uint32_t slot0 = base + rank_in(m0) + rank_in(m1);
    const uint32_t cs0 = cbase + incl - (k0 + k1);
    bool ovf = false;
    if (rect0) {
      if (slot0 < item_scap) {
        q_items[slot0] = Item{ptri, chan, sp.r0_start | (sp.r0_count << 16), pn};
        q_cs[slot0] = cs0;
      } else {
        ovf = true;
      }
    }
    if (rect1) {
      if (slot0 + 1u < item_scap) {
        q_items[slot0 + 1u] = Item{ptri, chan, sp.r1_start | (sp.r1_count << 16), pn};
        q_cs[slot0 + 1u] = cs0 + k0;
      } else {
        ovf = true;
      }
    }
    if (__ballot(ovf) != 0ull && lane == 0) atomicOr(&cnt->overflow, 1u);
  }
  if (lane == 0 && evaluated) atomicAdd(&cnt->items[shard].pairs, (unsigned long long)evaluated);
  if (lane == 0 && tested) atomicAdd(&cnt->items[shard].tests, (unsigned long long)tested);
  if (INLINE) {
    unsigned long long r = rtic;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) r += __shfl_xor(r, o, 64);
    if (lane == 0 && r) atomicAdd(&cnt->items[shard].rtic, r);
  }
}

// Intersection of the angular piece [p0, p1] (width <= 2 pi) with the arc
// [xl, xh] (width <= 2 pi): up to two pieces, written to (o0) and (o1).
__device__ inline void piece_cap_arc(bool pv, double p0, double p1, double xl, double xh,
                                     bool& v0, double& l0, double& h0, bool& v1, double& l1,
                                     double& h1) {
  v0 = v1 = false;
  l0 = h0 = l1 = h1 = 0.0;
  if (!pv) return;
  // shift the arc so that its start lies in (p0 - 2 pi, p0]; two copies cover P
  const double k = ceil((xl - p0) / TWO_PI);
  const double s0 = xl - k * TWO_PI, s1 = xh - k * TWO_PI;
  l0 = fmax(p0, s0); h0 = fmin(p1, s1); v0 = l0 <= h0;
  l1 = fmax(p0, s0 + TWO_PI); h1 = fmin(p1, s1 + TWO_PI); v1 = l1 <= h1;
}

// Ray-index ranges of one angular piece: (st0, ct0) and (st1, ct1), a count of
// 0 meaning no range.  Full-spin sensors wrap the index modulo chi; partial
// fields of view split a piece that runs past theta_0 + 2 pi.
__device__ inline void piece_ranges(const DevSensor& s, bool valid, double lo, double hi,
                                    uint32_t& st0, uint32_t& ct0, uint32_t& st1, uint32_t& ct1) {
  st0 = ct0 = st1 = ct1 = 0;
  if (!valid) return;
  // rays with azimuth offsets: nominal angle within max |offset| of the piece
  lo -= (double)s.az_noise;
  hi += (double)s.az_noise;
  const long chi = (long)s.chi;
  if (hi - lo >= TWO_PI) {
    ct0 = (uint32_t)chi;
    return;
  }
  double a = lo - s.theta_start_d;
  a -= TWO_PI * floor(a / TWO_PI);
  if (a < 0.0) a = 0.0;
  const double w = hi - lo;
  const double fa = a * s.inv_dtheta_d, fb = (a + w) * s.inv_dtheta_d;
  const long ra = (long)ceil(fa), rb = (long)floor(fb);
  if (s.wrap) {
    long c = rb - ra + 1;
    if (c > 0) {
      if (c > chi) c = chi;
      st0 = (uint32_t)(ra % chi);
      ct0 = (uint32_t)c;
    }
    return;
  }
  if (ra <= chi - 1 && rb >= ra) {
    const long e0 = rb < chi - 1 ? rb : chi - 1;
    st0 = (uint32_t)ra;
    ct0 = (uint32_t)(e0 - ra + 1);
  }
  const double fb2 = (a + w - TWO_PI) * s.inv_dtheta_d;
  if (fb2 >= 0.0) {
    long e1 = (long)floor(fb2);
    if (e1 > chi - 1) e1 = chi - 1;
    st1 = 0;
    ct1 = (uint32_t)(e1 + 1);
  }
}

// The candidate rays of channel (cj, sj): directions on the positive side
// of all three edge planes moved outward by SIN_M.  Each edge restricts the
// azimuth to an arc (or not at all, or completely); the pieces of their
// intersection are built with static slots (1 after the first arc, 2 after
// the second, 4 after the third) so that everything stays in registers.
struct ChannelPieces {
  bool whole;          // every azimuth is a candidate
  bool v[4];
  double lo[4], hi[4];
};

__device__ inline ChannelPieces channel_pieces(const double (&nrm)[3][3], const double (&beta)[3],
                                               const double (&hxy)[3], double cj, double sj) {
  ChannelPieces P;
  P.whole = true;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    P.v[i] = false;
    P.lo[i] = P.hi[i] = 0.0;
  }
  bool empty = false;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double Ak = fabs(cj) * hxy[k];
    const double rhs = -SIN_M - sj * nrm[k][2];
    if (empty || rhs <= -Ak) continue;  // this edge keeps every azimuth
    if (rhs > Ak) {                     // this edge keeps none
      empty = true;
      continue;
    }
    const double rho = fmin(1.0, fmax(-1.0, rhs / Ak));
    const double wd = acos(rho);
    // cos(phi) < 0 (a channel rounded past the pole) mirrors the azimuth
    const double bc = cj >= 0.0 ? beta[k] : beta[k] + 3.14159265358979323846;
    const double xl = bc - wd, xh = bc + wd;
    if (P.whole) {
      P.whole = false;
      P.v[0] = true; P.lo[0] = xl; P.hi[0] = xh;
    } else if (k == 1) {
      bool v0, v1;
      double l0, h0, l1, h1;
      piece_cap_arc(P.v[0], P.lo[0], P.hi[0], xl, xh, v0, l0, h0, v1, l1, h1);
      P.v[0] = v0; P.lo[0] = l0; P.hi[0] = h0;
      P.v[1] = v1; P.lo[1] = l1; P.hi[1] = h1;
    } else if (k == 2) {
      bool v0, v1, v2, v3;
      double l0, h0, l1, h1, l2, h2, l3, h3;
      piece_cap_arc(P.v[0], P.lo[0], P.hi[0], xl, xh, v0, l0, h0, v1, l1, h1);
      piece_cap_arc(P.v[1], P.lo[1], P.hi[1], xl, xh, v2, l2, h2, v3, l3, h3);
      P.v[0] = v0; P.lo[0] = l0; P.hi[0] = h0;
      P.v[1] = v1; P.lo[1] = l1; P.hi[1] = h1;
      P.v[2] = v2; P.lo[2] = l2; P.hi[2] = h2;
      P.v[3] = v3; P.lo[3] = l3; P.hi[3] = h3;
    }
  }
  if (empty) {
    P.whole = false;
#pragma unroll
    for (int i = 0; i < 4; ++i) P.v[i] = false;
  }
  return P;
}

// The shards a persistent consumer wave serves: shard (global wave index mod
// NSHARD), or, on a grid of fewer than NSHARD waves, every shard congruent to
// the wave index.  Each shard is drained by its own waves through the shard's
// ticket, so no counter is shared by more than a few dozen waves.
struct ShardWalk {
  uint32_t first, step, nw;  // nw: waves in the grid
};

__device__ inline ShardWalk shard_walk(uint32_t wpb) {
  const uint32_t gw = blockIdx.x * wpb + wave_id();
  const uint32_t nw = gridDim.x * wpb;
  const uint32_t step = nw < NSHARD ? nw : NSHARD;
  return ShardWalk{gw % step, step, nw};
}

// One wave per large-class record: lanes take the record's channels, 64 at a
// time; each lane intersects the azimuth arcs of the three edge planes on its
// channel and emits the resulting ray ranges, chopped into row items of at
// most row_chunk rays, to an item shard of the lane's own.
template <int WPB>
__global__ __launch_bounds__(WPB * 64) void expand_kernel(
    const DevScene* __restrict__ scenes, const DevSensor* __restrict__ sens,
    const Item* __restrict__ large, Item* __restrict__ items, uint32_t* __restrict__ item_cs,
    uint32_t item_scap, uint32_t large_scap, uint32_t row_chunk, Counters* __restrict__ cnt) {
  const uint32_t lane = lane_id();
  const ShardWalk sw = shard_walk(WPB);
  uint32_t rows = 0;  // row items this wave appended (statistic)
  // Each lane appends its channel's rows to an item shard of its own, the
  // lanes of a batch to consecutive shards from s0, which moves on past them
  // with every batch: one record near a sensor can hold hundreds of
  // thousands of candidates, and they are spread over all shards.
  uint32_t s0 = sw.first;
  // records dealt statically: the waves walking a shard take every
  // walkers-th record from their rank (no ticket round trip; a record's
  // work varies little)
  const uint32_t gw = blockIdx.x * WPB + wave_id();
  const uint32_t rank = gw / sw.step;
  const uint32_t walkers = (gridDim.x * WPB - sw.first + sw.step - 1u) / sw.step;
  for (uint32_t sh = sw.first; sh < NSHARD; sh += sw.step) {
    const uint32_t n_large = min((uint32_t)cnt->large[sh].nc, large_scap);
    const Item* const q_large = large + (size_t)sh * large_scap;
    for (uint32_t rec = rank; rec < n_large; rec += walkers) {
      const Item L = q_large[rec];
      const DevSensor& s = sens[L.sensor];
      const DevScene& S = scenes[s.scene];
      const uint32_t t = L.tri;
      // a static triangle's vertex records in one round trip
      float4 p0, p1, p2;
      if (t < S.n_soup) {
        p0 = S.soup[3ull * t];
        p1 = S.soup[3ull * t + 1];
        p2 = S.soup[3ull * t + 2];
      } else {
        const uint32_t i0 = S.idx[3ull * t], i1 = S.idx[3ull * t + 1], i2 = S.idx[3ull * t + 2];
        p0 = S.v[i0];
        p1 = S.v[i1];
        p2 = S.v[i2];
      }
      Statics st;
      double nrm[3][3];
      if (!make_statics(p0.x, p0.y, p0.z, p1.x, p1.y, p1.z, p2.x, p2.y, p2.z, s, st, nrm))
        continue;
      // the three edge planes' angles, lane k computing edge k (one atan2
      // and one sqrt in the instruction stream instead of three each; the
      // values are the same), then read from lanes 0-2
      const uint32_t ke = lane < 3u ? lane : 0u;
      const double ex = ke == 0u ? nrm[0][0] : (ke == 1u ? nrm[1][0] : nrm[2][0]);
      const double ey = ke == 0u ? nrm[0][1] : (ke == 1u ? nrm[1][1] : nrm[2][1]);
      const double be = atan2(ey, ex);
      const double he = sqrt(ex * ex + ey * ey);
      double beta[3], hxy[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        beta[k] = lane_f64(be, k);
        hxy[k] = lane_f64(he, k);
      }
      const uint32_t c_from = L.chan & 0xFFFFu, c_count = L.chan >> 16;
      for (uint32_t base = 0; base < c_count; base += 64) {
        const uint32_t j = c_from + base + lane;
        const bool act = base + lane < c_count;
        // up to 4 pieces x 2 index ranges per channel, in fixed slots
        uint32_t rs[8], rc[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) rs[i] = rc[i] = 0;
        if (act) {
          const double2 cs = s.chan_d[j];
          const ChannelPieces P = channel_pieces(nrm, beta, hxy, cs.x, cs.y);
          if (P.whole) {
            rc[0] = s.chi;
          } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
              piece_ranges(s, P.v[i], P.lo[i], P.hi[i], rs[2 * i], rc[2 * i], rs[2 * i + 1],
                           rc[2 * i + 1]);
          }
        }
        // count row items (ranges chopped into row_chunk rays) and their candidates
        uint32_t nitems = 0, ncand = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          nitems += (rc[i] + row_chunk - 1) / row_chunk;
          ncand += rc[i];
        }
        const unsigned long long mine = __ballot(nitems != 0u);
        if (mine == 0ull) continue;
        const uint32_t osh = (s0 + rank_in(mine)) % NSHARD;
        s0 = (s0 + (uint32_t)__popcll(mine)) % NSHARD;
        if (nitems == 0u) continue;
        // (at most 8 ranges of at most chi < 2^16 rays per channel)
        const unsigned long long old = atomicAdd(
            &cnt->items[osh].nc, (unsigned long long)nitems | ((unsigned long long)ncand << 32));
        rows += nitems;
        uint32_t slot = (uint32_t)old;
        uint32_t cs = (uint32_t)(old >> 32);
        if (cs > CAND_LIMIT - ncand) atomicOr(&cnt->overflow, 4u);
        Item* const q_items = items + (size_t)osh * item_scap;
        uint32_t* const q_cs = item_cs + (size_t)osh * item_scap;
        bool ovf = false;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          for (uint32_t o = 0; o < rc[i]; o += row_chunk) {
            const uint32_t c = min(row_chunk, rc[i] - o);
            uint32_t r0 = rs[i] + o;
            if (r0 >= s.chi) r0 -= s.chi;
            if (slot < item_scap) {
              q_items[slot] = Item{t, j | (1u << 16), r0 | (c << 16), L.sensor};
              q_cs[slot] = cs;
            } else {
              ovf = true;
            }
            ++slot;
            cs += c;
          }
        }
        if (ovf) atomicOr(&cnt->overflow, 1u);
      }
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) rows += __shfl_xor(rows, o, 64);
  if (lane == 0 && rows) atomicAdd(&cnt->items[sw.first].rows, rows);
}

// ------------------------------------------------------------------ intersection
// LDS record of a staged item (24 B; its statics' twelve normal components
// sit in a separate array of float4s).
struct ItemInfo {
  uint32_t tri;
  uint32_t cr;    // c_from | r_start << 16
  uint32_t rs;    // r_count | sensor slot << 16
  int32_t bias;   // item-local candidate index = batch position + bias
  float inv_rc;   // 1 / r_count
  float h;        // origin-to-plane distance of the statics
};

// What the intersection needs of a sensor and its scene, cached in LDS for
// the first 64 sensor slots of the cast.
struct IsectSensor {
  const float2* chan;
  const float2* az;
  const uint8_t* mask;
  const uint32_t* idx;
  const uint32_t* orig;
  const float4* v;
  const float4* soup;
  uint32_t n_soup;
  float o[3], f[3], r[3], u[3];
  int32_t cull_back;
  uint32_t chi, key_offset;
  float dmin, dmax;
};

__device__ inline IsectSensor isect_sensor(const DevScene* scenes, const DevSensor& s) {
  const DevScene& S = scenes[s.scene];
  IsectSensor q;
  q.chan = s.chan; q.az = s.az; q.mask = s.mask;
  q.idx = S.idx; q.orig = S.orig; q.v = S.v; q.soup = S.soup; q.n_soup = S.n_soup;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    q.o[k] = s.o[k]; q.f[k] = s.f[k]; q.r[k] = s.r[k]; q.u[k] = s.u[k];
  }
  q.cull_back = s.cull_back;
  q.chi = s.chi; q.key_offset = s.key_offset; q.dmin = s.dmin; q.dmax = s.dmax;
  return q;
}

// The sensor fields the candidate loop keeps in registers.
struct CandSensor {
  const float2* chan;
  const float2* az;
  const uint8_t* mask;
  uint32_t chi, key_offset;
  float dmin, dmax;
};

// Item i of a wave's staged ItemInfo array in LDS, read through an LDS
// pointer so that the address is 32-bit arithmetic (a generic pointer would
// make it a 64-bit multiply-add).
__device__ inline ItemInfo lds_item(const ItemInfo* base, uint32_t i) {
  typedef const uint32_t __attribute__((address_space(3))) LU;
  typedef const char __attribute__((address_space(3))) LC;
  static_assert(sizeof(ItemInfo) == 24, "six words");
  LU* p = (LU*)((LC*)base + __umul24(24u, i));
  ItemInfo o;
  o.tri = p[0];
  o.cr = p[1];
  o.rs = p[2];
  o.bias = (int32_t)p[3];
  o.inv_rc = __uint_as_float(p[4]);
  o.h = __uint_as_float(p[5]);
  return o;
}

// One candidate of the flattened loop, from its owner item (staged in LDS)
// and batch position f: the ray's table entries and the ray's key as this
// wave can see it, all reads issued together.  The key is read atomically
// (relaxed), so it is some value the key held: never below the true minimum,
// since keys only decrease.  A hit that is not below it cannot improve on the
// final key and skips its atomic; the atomicMin stays the authority.  The
// owner's statics are read from LDS when the candidate is tested, so that a
// lane can keep several candidates in flight.
struct Cand {
  float2 cp, ca;
  unsigned long long seen;
  uint32_t kidx;
  bool on;  // the ray is active (mask)
};
// LDS_SENS: every sensor slot of the cast is below 64 and read from the
// block's LDS copy; otherwise from the device descriptors.  (One source per
// instance: a per-lane choice between the two would turn every read into a
// flat access, which also waits behind the LDS counter.)
template <bool LDS_SENS>
__device__ inline CandSensor cand_sensor(uint32_t sid, const IsectSensor* sen,
                                         const DevSensor* sens) {
  if (LDS_SENS) {
    const IsectSensor& q = sen[sid];
    return CandSensor{q.chan, q.az, q.mask, q.chi, q.key_offset, q.dmin, q.dmax};
  }
  const DevSensor& q = sens[sid];
  return CandSensor{q.chan, q.az, q.mask, q.chi, q.key_offset, q.dmin, q.dmax};
}
template <bool LDS_SENS>
__device__ inline Cand cand_read(int own, uint32_t f, const ItemInfo* in_w,
                                 const IsectSensor* sen, const DevSensor* sens,
                                 const unsigned long long* keys, bool any_mask) {
  const ItemInfo inf = lds_item(in_w, (uint32_t)own);
  const CandSensor sn = cand_sensor<LDS_SENS>(inf.rs >> 16, sen, sens);
  // batch position -> (channel, ray) of the item's rectangle.  local is
  // below 255 x 65535 < 2^24 (the span-class limits), so it is exact in
  // FP32 and local x rcp(r_count) is within 1 of the quotient for r_count
  // >= 3 (exact for 1 and 2); one correction step makes it exact.  Every
  // product below stays under 2^25: 24-bit multiplies.
  const uint32_t r_count = inf.rs & 0xFFFFu;
  const uint32_t local = (uint32_t)((int32_t)f + inf.bias);
  // within 1 of the quotient (0 for local < r_count); two branch-free
  // corrections make it exact
  uint32_t c = (uint32_t)((float)local * inf.inv_rc);
  c -= (uint32_t)(__umul24(c, r_count) > local);
  c += (uint32_t)(__umul24(c + 1u, r_count) <= local);
  const uint32_t r = local - __umul24(c, r_count);
  const uint32_t ch = (inf.cr & 0xFFFFu) + c;
  uint32_t ray = (inf.cr >> 16) + r;
  if (ray >= sn.chi) ray -= sn.chi;
  const uint32_t gl = __umul24(ch, sn.chi) + ray;
  Cand o;
  o.on = true;
  if (any_mask) o.on = !sn.mask || gload(sn.mask, gl);
  o.cp = gload_f2(sn.chan, ch * 8u);
  o.ca = gload_f2(sn.az, ray * 8u);
  o.kidx = sn.key_offset + gl;
  // a single-copy-atomic read: another wave's atomicMin may land at any time.
  // Workgroup scope lets it hit a stale cache line; keys only decrease, so a
  // stale value is never below the current one and only costs a redundant atomic.
  o.seen = __hip_atomic_load(const_cast<unsigned long long*>(keys) + o.kidx, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
  return o;
}
// The ray test against the owner's statics, and the atomic for a hit that
// can improve on the key read (returns whether one was issued).
template <bool LDS_SENS>
__device__ inline uint32_t cand_finish(const Cand& o, int own, const float4 (*st_w)[64],
                                   const ItemInfo* in_w, const IsectSensor* sen,
                                   const DevSensor* sens, unsigned long long* keys) {
  const uint32_t ow = (uint32_t)own;
  const ItemInfo inf = lds_item(in_w, ow);
  const float4 a0 = st_w[0][ow], a1 = st_w[1][ow], a2 = st_w[2][ow];
  const Statics st{a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w,
                   a2.x, a2.y, a2.z, a2.w, inf.h, 0.0f, 0.0f, 0.0f};
  const uint32_t sid = inf.rs >> 16;
  const float dmin = LDS_SENS ? sen[sid].dmin : sens[sid].dmin;
  const float dmax = LDS_SENS ? sen[sid].dmax : sens[sid].dmax;
  const unsigned long long key = ray_test(st, o.cp.x, o.cp.y, o.ca.x, o.ca.y, dmin, dmax, inf.tri);
  if (o.on && key < o.seen) {
    key_min(keys, o.kidx, key);
    return 1u;
  }
  return 0u;
}

// Inclusive prefix maximum over the wave of values >= 0, by DPP row shifts
// and row broadcasts (no LDS round trips).  0 is the identity: lanes without
// a source (bound_ctrl) and the rows a broadcast leaves out read 0, so each
// step folds into one max instruction.
__device__ inline uint32_t wave_incl_max0(uint32_t v) {
#define GRCA_MAX0_STEP(CTRL, ROWS) \
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, true));
  GRCA_MAX0_STEP(0x111, 0xf)  // row_shr:1
  GRCA_MAX0_STEP(0x112, 0xf)  // row_shr:2
  GRCA_MAX0_STEP(0x114, 0xf)  // row_shr:4
  GRCA_MAX0_STEP(0x118, 0xf)  // row_shr:8
  GRCA_MAX0_STEP(0x142, 0xa)  // row_bcast:15
  GRCA_MAX0_STEP(0x143, 0xc)  // row_bcast:31
#undef GRCA_MAX0_STEP
  return v;
}

// Last slot i in [0, n) of a shard with cs[i] <= a (cs increasing, cs[0] = 0
// <= a): a 64-way search, one probe per lane per round.
__device__ inline uint32_t find_owner(const uint32_t* __restrict__ cs, uint32_t n, uint32_t a) {
  const uint32_t lane = lane_id();
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1u) {
    const uint32_t step = (hi - lo + 63u) / 64u;
    const uint32_t p = lo + lane * step;
    const bool le = p < hi && cs[p] <= a;  // lane 0 probes lo: always true
    const unsigned long long m = __ballot(le);
    lo += (uint32_t)(63 - __clzll((long long)m)) * step;
    hi = min(lo + step, hi);
  }
  return lo;
}

// Persistent intersection with candidate-balanced tickets.  Every queued item
// knows the index of its first candidate pair within its shard, so a ticket
// is a fixed range [a, b) of candidate pairs: the wave finds the item holding
// candidate a, then stages the items overlapping [a, b) 64 at a time (lane k
// gathers item k's triangle, builds the pair's FP64 statics and keeps them
// with the sensor fields in LDS, clipped to the ticket) and walks the
// FLATTENED list of their candidates, 64 pairs per step.  Every ticket costs
// the same whatever the sizes of the items in it.  Invalid pairs (degenerate,
// or back-facing under single-sided casting) contribute no candidates.
// Candidates per lane per window of the intersection's flattened loop: 4
// keeps it under 128 VGPRs (4 waves per SIMD) and measured 0.259 ms against
// 0.263 ms for 2 and 0.282 ms for 6 (3 waves per SIMD) on the ring workload.
constexpr int ISECT_SLOTS = 4;
// A shard's last (waves serving it) x ticket_cands candidates are handed out
// in tickets of ticket_cands / TAIL_DIV, so that its waves run out of work
// within a short ticket of each other instead of a long one: with tickets of
// 4096, intersection 0.190 -> 0.178 ms on the ring workload.
constexpr uint32_t TAIL_DIV = 4;
template <int WPB, bool LDS_SENS>
__global__ __launch_bounds__(WPB * 64) void isect_kernel(
    const DevScene* __restrict__ scenes, const DevSensor* __restrict__ sens,
    uint32_t nsens, const Item* __restrict__ items, const uint32_t* __restrict__ item_cs,
    uint32_t item_scap, uint32_t ticket_cands, Counters* __restrict__ cnt,
    unsigned long long* __restrict__ keys) {
  __shared__ float4 st_s[WPB][3][64];  // the staged items' normals n0, n1, n2, N
  __shared__ ItemInfo in_s[WPB][64];
  __shared__ uint32_t mark_s[WPB][64 * ISECT_SLOTS];  // owner + 1 at its first position, else 0
  __shared__ IsectSensor sen_s[64];
  const uint32_t w = wave_id();
  const uint32_t lane = lane_id();
  if (LDS_SENS && threadIdx.x < nsens) sen_s[threadIdx.x] = isect_sensor(scenes, sens[threadIdx.x]);
  // whether any sensor of the cast has an active-ray mask (block-uniform)
  bool has_mask = false;
  for (uint32_t k = threadIdx.x; k < nsens; k += blockDim.x) has_mask |= sens[k].mask != nullptr;
  const bool any_mask = __syncthreads_or(has_mask) != 0;
  const ShardWalk sw = shard_walk(WPB);
  unsigned long long rtic = 0ull;  // wave-uniform
  uint32_t natom = 0;              // atomic minima this lane issued
  for (uint32_t sh = sw.first; sh < NSHARD; sh += sw.step) {
    const unsigned long long nc = cnt->items[sh].nc;
    const uint32_t n_items = min((uint32_t)nc, item_scap);
    const uint32_t n_cand = (uint32_t)(nc >> 32);
    if (n_items == 0u || n_cand > CAND_LIMIT) continue;  // the latter is reported as overflow
    const size_t off = (size_t)sh * item_scap;
    const Item* const q = items + off;
    const uint32_t* const qcs = item_cs + off;
    // Ticket k (the shard's ticket counter counts tickets): candidates
    // [k t, (k + 1) t) while they end before the shard's tail, the last
    // (waves serving the shard) x t candidates; the tail in tickets of
    // t / TAIL_DIV (t = ticket_cands).
    const uint32_t n_waves = sw.step < NSHARD ? 1u : (sw.nw - sh + NSHARD - 1u) / NSHARD;
    const uint32_t t_tail = max(ticket_cands / TAIL_DIV, 64u);
    const uint32_t tail = (uint32_t)min<uint64_t>((uint64_t)n_waves * ticket_cands, n_cand);
    const uint32_t n_big = (n_cand - tail) / ticket_cands;
    const uint32_t big_end = n_big * ticket_cands;
    for (;;) {
      uint32_t k = 0;
      if (lane == 0) k = atomicAdd(&cnt->items[sh].tk, 1u);
      k = first_lane(k);
      uint32_t a, b;
      if (k < n_big) {
        a = k * ticket_cands;
        b = a + ticket_cands;
      } else {
        const uint64_t a64 = (uint64_t)big_end + (uint64_t)(k - n_big) * t_tail;
        if (a64 >= n_cand) break;
        a = (uint32_t)a64;
        b = n_cand - a > t_tail ? a + t_tail : n_cand;
      }
      uint32_t ib = find_owner(qcs, n_items, a);
      // the stage's items and their first candidate indices; each stage
      // issues the next stage's reads before its candidate windows
      uint32_t nc0 = 0xFFFFFFFFu;
      Item nit{};
      if (ib + lane < n_items) {
        nc0 = qcs[ib + lane];
        nit = q[ib + lane];
      }
      for (; ib < n_items; ib += 64u) {
        const uint32_t i = ib + lane;
        uint32_t count = 0, skip = 0;
        const uint32_t c0 = nc0;
        const Item it = nit;
        const bool past = i >= n_items || c0 >= b;  // this lane's item starts at or after b
        if (!past) {
          const uint32_t rc = it.rays >> 16;
          const uint64_t e = (uint64_t)c0 + (uint64_t)((it.chan >> 16) * rc);
          const uint32_t lo = max(c0, a);
          const uint32_t hi = (uint32_t)min<uint64_t>(e, (uint64_t)b);
          if (hi > lo) {
            // the pair's statics, built here in FP64 from the gathered triangle
            const IsectSensor sq = LDS_SENS ? sen_s[it.sensor]
                                            : isect_sensor(scenes, sens[it.sensor]);
            // (global loads at 32-bit byte offsets: the pointers come from
            // LDS, and flat accesses would also wait behind the LDS counter)
            // (a static triangle's vertex records in one round trip)
            const uint32_t t = it.tri;
            float4 p0, p1, p2;
            if (t < sq.n_soup) {
              p0 = gload_v(sq.soup, 48u * t);
              p1 = gload_v(sq.soup, 48u * t + 16u);
              p2 = gload_v(sq.soup, 48u * t + 32u);
            } else {
              const Tri3 ti = gload_tri(sq.idx, 12u * t);
              p0 = gload_v(sq.v, 16u * ti.a);
              p1 = gload_v(sq.v, 16u * ti.b);
              p2 = gload_v(sq.v, 16u * ti.c);
            }
            Statics st;
            if (make_statics(p0.x, p0.y, p0.z, p1.x, p1.y, p1.z, p2.x, p2.y, p2.z, sq, st)) {
              count = hi - lo;
              st_s[w][0][lane] = make_float4(st.n0x, st.n0y, st.n0z, st.n1x);
              st_s[w][1][lane] = make_float4(st.n1y, st.n1z, st.n2x, st.n2y);
              st_s[w][2][lane] = make_float4(st.n2z, st.Nx, st.Ny, st.Nz);
              ItemInfo inf;
              inf.tri = gload(sq.orig, 4u * it.tri);  // keys carry the caller's triangle id
              inf.cr = (it.chan & 0xFFFFu) | (it.rays << 16);
              inf.rs = rc | (it.sensor << 16);
              inf.bias = 0;
              inf.inv_rc = __builtin_amdgcn_rcpf((float)rc);  // an estimate: corrected below
              inf.h = st.h;
              in_s[w][lane] = inf;
              skip = lo - c0;  // candidates of the item before this ticket
            }
          }
        }
        const bool last = __ballot(past) != 0ull;
        nc0 = 0xFFFFFFFFu;
        nit = Item{};
        if (!last && i + 64u < n_items) {
          nc0 = qcs[i + 64u];
          nit = q[i + 64u];
        }
        const uint32_t incl = wave_incl_scan(count);
        const uint32_t excl = incl - count;  // batch position of this item's first candidate
        if (count) in_s[w][lane].bias = (int32_t)skip - (int32_t)excl;
        const uint32_t total = last_lane(incl);
        rtic += total;
        // Owner of batch position p: the last item with a candidate whose first
        // position is <= p.  Per window of 64 x ISECT_SLOTS positions, each
        // item starting in the window marks its slot, and a prefix maximum
        // spreads the marks; positions before the first mark keep the
        // previous window's owner.  Each lane takes the positions p + 64 j:
        // all its candidates' table and key reads are in flight together.
        constexpr uint32_t WIN = 64u * ISECT_SLOTS;
        uint32_t carry = 0;  // owner + 1 of the position before the window
        for (uint32_t base = 0; base < total; base += WIN) {
#pragma unroll
          for (int j = 0; j < ISECT_SLOTS; ++j) mark_s[w][64 * j + lane] = 0u;
          wave_sync();
          if (count && excl >= base && excl - base < WIN) mark_s[w][excl - base] = lane + 1u;
          wave_sync();
          int own[ISECT_SLOTS];
#pragma unroll
          for (int j = 0; j < ISECT_SLOTS; ++j) {
            const uint32_t o1 = max(wave_incl_max0(mark_s[w][64 * j + lane]), carry);
            carry = (uint32_t)__builtin_amdgcn_readlane((int)o1, 63);
            own[j] = (int)o1 - 1;
          }
          wave_sync();
          if (base + lane >= total) continue;  // and every later position
          Cand c[ISECT_SLOTS];
#pragma unroll
          for (int j = 0; j < ISECT_SLOTS; ++j)
            if (j == 0 || base + 64u * j + lane < total)
              c[j] = cand_read<LDS_SENS>(own[j], base + 64u * j + lane, in_s[w], sen_s, sens, keys,
                                         any_mask);
#pragma unroll
          for (int j = 0; j < ISECT_SLOTS; ++j)
            if (j == 0 || base + 64u * j + lane < total)
              natom += cand_finish<LDS_SENS>(c[j], own[j], st_s[w], in_s[w], sen_s, sens, keys);
        }
        wave_sync();
        if (last) break;
      }
    }
  }
  if (lane == 0 && rtic) atomicAdd(&cnt->items[sw.first].rtic, rtic);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) natom += __shfl_xor(natom, o, 64);
  if (lane == 0 && natom) atomicAdd(&cnt->items[sw.first].atomics, (unsigned long long)natom);
}

// ------------------------------------------------------------------ all pairs
__global__ void statics_kernel(const DevScene* __restrict__ scenes, const DevSensor* __restrict__ sens,
                               uint32_t sensor, Statics* __restrict__ out) {
  const DevSensor& s = sens[sensor];
  const DevScene& S = scenes[s.scene];
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= S.ntri) return;
  const uint32_t i0 = S.idx[3ull * t], i1 = S.idx[3ull * t + 1], i2 = S.idx[3ull * t + 2];
  const float4 p0 = S.v[i0], p1 = S.v[i1], p2 = S.v[i2];
  Statics st;
  if (!make_statics(p0.x, p0.y, p0.z, p1.x, p1.y, p1.z, p2.x, p2.y, p2.z, s, st)) {
    st = Statics{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, -1.0f, 0, 0, 0};
  }
  out[S.orig[t]] = st;  // the all-pairs pass walks the caller's triangle ids
}

// One thread per ray, loop over a chunk of triangles; every ray is tested
// against every triangle of the chunk.
__global__ __launch_bounds__(256) void allpairs_kernel(const DevSensor* __restrict__ sens,
                                                       uint32_t sensor, const Statics* __restrict__ st_all,
                                                       uint32_t ntri, uint32_t chunk,
                                                       unsigned long long* __restrict__ keys) {
  __shared__ Statics tile[256];
  const DevSensor& s = sens[sensor];
  const uint32_t nrays = s.gamma * s.chi;
  const uint32_t g = blockIdx.x * 256 + threadIdx.x;
  const bool act = g < nrays && !(s.mask && !s.mask[g]);
  const uint32_t ch = act ? g / s.chi : 0, ray = act ? g % s.chi : 0;
  const float2 cp = s.chan[ch];
  const float2 ca = s.az[ray];
  unsigned long long best = KEY_INIT;
  const uint32_t t_begin = blockIdx.y * chunk;
  const uint32_t t_end = min(ntri, t_begin + chunk);
  for (uint32_t t0 = t_begin; t0 < t_end; t0 += 256) {
    __syncthreads();
    if (t0 + threadIdx.x < t_end) tile[threadIdx.x] = st_all[t0 + threadIdx.x];
    __syncthreads();
    const uint32_t n = min(256u, t_end - t0);
    if (act) {
      for (uint32_t k = 0; k < n; ++k) {
        const unsigned long long key =
            ray_test(tile[k], cp.x, cp.y, ca.x, ca.y, s.dmin, s.dmax, t0 + k);
        best = key < best ? key : best;
      }
    }
  }
  if (act && best != KEY_INIT) key_min(keys, s.key_offset + g, best);
}

// ------------------------------------------------------------------ resolve
template <bool VEC>
__global__ void resolve_kernel(const unsigned long long* __restrict__ keys, uint32_t n,
                               float* __restrict__ dist, uint32_t* __restrict__ tri,
                               Counters* __restrict__ cnt) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x < 64) {
    // the cast's summary: totals and per-shard maxima of the queue counters
    const uint32_t l = threadIdx.x;
    uint32_t ni = (uint32_t)cnt->items[l].nc, nl = (uint32_t)cnt->large[l].nc;
    uint32_t nr = cnt->items[l].rows;
    unsigned long long rt = cnt->items[l].rtic, pr = cnt->items[l].pairs;
    unsigned long long te = cnt->items[l].tests, at = cnt->items[l].atomics;
    uint32_t mi = ni, ml = nl;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      ni += __shfl_xor(ni, o, 64);
      nl += __shfl_xor(nl, o, 64);
      nr += __shfl_xor(nr, o, 64);
      rt += __shfl_xor(rt, o, 64);
      pr += __shfl_xor(pr, o, 64);
      te += __shfl_xor(te, o, 64);
      at += __shfl_xor(at, o, 64);
      mi = max(mi, (uint32_t)__shfl_xor(mi, o, 64));
      ml = max(ml, (uint32_t)__shfl_xor(ml, o, 64));
    }
    if (l == 0) {
      Summary& S = cnt->sum;
      S.n_items = ni; S.n_large = nl; S.n_rows = nr; S.overflow = cnt->overflow;
      S.max_items_shard = mi; S.max_large_shard = ml; S.rtic = rt; S.pairs = pr;
      S.tests = te;
      S.atomics = at;
      Sticky k = cnt->sticky;
      if (cnt->overflow) {
        k.overflow |= cnt->overflow;
        k.casts += 1u;
        k.max_items_shard = max(k.max_items_shard, mi);
        k.max_large_shard = max(k.max_large_shard, ml);
        cnt->sticky = k;
      }
      S.sticky = k;
    }
  }
  // rays 4g .. 4g + 3: 16-byte loads and stores when the outputs allow them
  const uint32_t r0 = 4u * g;
  if (r0 >= n) return;
  const bool vec = VEC && r0 + 3u < n;
  unsigned long long k[4];
  if (vec) {
    const ulonglong2* p = reinterpret_cast<const ulonglong2*>(keys + r0);
    const ulonglong2 a = p[0], b = p[1];
    k[0] = a.x; k[1] = a.y; k[2] = b.x; k[3] = b.y;
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) k[j] = r0 + j < n ? keys[r0 + j] : KEY_INIT;
  }
  float d[4];
  uint32_t t[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t hi = (uint32_t)(k[j] >> 32);
    // inverse of f_sort: m = ((u >> 31) - 1) | 2^31
    const uint32_t m = ((hi >> 31) - 1u) | 0x80000000u;
    d[j] = __uint_as_float(hi ^ m);
    t[j] = (uint32_t)k[j];
  }
  if (vec) {
    if (dist) *reinterpret_cast<float4*>(dist + r0) = make_float4(d[0], d[1], d[2], d[3]);
    if (tri) *reinterpret_cast<uint4*>(tri + r0) = make_uint4(t[0], t[1], t[2], t[3]);
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (r0 + j >= n) break;
      if (dist) dist[r0 + j] = d[j];
      if (tri) tri[r0 + j] = t[j];
    }
  }
}

// ------------------------------------------------------------------ pose
// One launch for both kinds: blocks [0, n_rigid) are rigid-instance blocks,
// the rest deform-group blocks; each thread poses the block's vertices
// i, i + 256, i + 512 and i + 768 (their loads in flight together).
__global__ __launch_bounds__(256) void pose_kernel(
    const PoseBlock* __restrict__ rblocks, uint32_t n_rigid, const float* __restrict__ rrx,
    const float* __restrict__ rry, const float* __restrict__ rrz,
    const PoseBlock* __restrict__ dblocks, const float* __restrict__ drx,
    const float* __restrict__ dry, const float* __restrict__ drz, const float* __restrict__ nx,
    const float* __restrict__ ny, const float* __restrict__ nz, const float* __restrict__ phase,
    const DeformParam* __restrict__ groups, const double* __restrict__ pose_in,
    float4* __restrict__ out) {
  constexpr uint32_t PER = POSE_BLOCK_VERTS / 256;
  const bool rigid = blockIdx.x < n_rigid;
  const PoseBlock pb = rigid ? rblocks[blockIdx.x] : dblocks[blockIdx.x - n_rigid];
  if (rigid) {
    const float* M = reinterpret_cast<const float*>(pose_in + 1) + 12ull * pb.group;
    float x[PER], y[PER], z[PER];
#pragma unroll
    for (uint32_t k = 0; k < PER; ++k) {  // (clamped: every load in bounds, all in flight)
      const uint32_t r = pb.rest_begin + min(threadIdx.x + 256u * k, pb.count - 1u);
      x[k] = rrx[r]; y[k] = rry[r]; z[k] = rrz[r];
    }
#pragma unroll
    for (uint32_t k = 0; k < PER; ++k) {
      const uint32_t i = threadIdx.x + 256u * k;
      if (i >= pb.count) break;
      const double px = x[k], py = y[k], pz = z[k];
      out[pb.v_begin + i] = make_float4(
          (float)((double)M[0] * px + (double)M[1] * py + (double)M[2] * pz + (double)M[3]),
          (float)((double)M[4] * px + (double)M[5] * py + (double)M[6] * pz + (double)M[7]),
          (float)((double)M[8] * px + (double)M[9] * py + (double)M[10] * pz + (double)M[11]),
          0.0f);
    }
  } else {
    const DeformParam g = groups[pb.group];
    const double time = pose_in[0];
    float x[PER], y[PER], z[PER], ux[PER], uy[PER], uz[PER], ph[PER];
#pragma unroll
    for (uint32_t k = 0; k < PER; ++k) {  // (clamped: every load in bounds, all in flight)
      const uint32_t r = pb.rest_begin + min(threadIdx.x + 256u * k, pb.count - 1u);
      x[k] = drx[r]; y[k] = dry[r]; z[k] = drz[r];
      ux[k] = nx[r]; uy[k] = ny[r]; uz[k] = nz[r]; ph[k] = phase[r];
    }
#pragma unroll
    for (uint32_t k = 0; k < PER; ++k) {
      const uint32_t i = threadIdx.x + 256u * k;
      if (i >= pb.count) break;
      const double wv = (double)g.amplitude * sin((double)g.omega * time + (double)ph[k]);
      out[pb.v_begin + i] = make_float4((float)((double)x[k] + wv * (double)ux[k]),
                                        (float)((double)y[k] + wv * (double)uy[k]),
                                        (float)((double)z[k] + wv * (double)uz[k]), 0.0f);
    }
  }
}

// ------------------------------------------------------------------ sensor tables
__global__ void sensor_tables_kernel(const float* __restrict__ elev, const float* __restrict__ el_off,
                                     uint32_t gamma, uint32_t chi, double dtheta,
                                     const float* __restrict__ az_off, float2* __restrict__ chan,
                                     double2* __restrict__ chan_d, float* __restrict__ sin_tab,
                                     float2* __restrict__ az) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < gamma) {
    // the nominal elevation for the channel search, the perturbed one
    // (vertical noise) for the rays
    const double p = (double)elev[i];
    const double q = el_off ? p + (double)el_off[i] : p;
    const double c = cos(q), s = sin(q);
    chan[i] = make_float2((float)c, (float)s);
    chan_d[i] = make_double2(c, s);
    sin_tab[i] = (float)sin(p);
  }
  if (i < chi) {
    // theta_R = (R - floor(chi / 2)) * dtheta (section 3.1, centred start)
    double th = ((double)i - (double)(chi / 2)) * dtheta;
    if (az_off) th += (double)az_off[i];
    az[i] = make_float2((float)cos(th), (float)sin(th));
  }
}

__global__ void sensor_lut_kernel(const float* __restrict__ sin_tab, uint32_t gamma,
                                  uint32_t lut_size, ChanBin* __restrict__ bins) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= lut_size) return;
  const float edge = -1.0f + 2.0f * (float)b / (float)lut_size;
  uint32_t lo = 0, hi = gamma;  // first j with sin_tab[j] >= edge
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (sin_tab[mid] < edge) lo = mid + 1; else hi = mid;
  }
  const float inf = __builtin_huge_valf();
  ChanBin e;
  e.j = lo;
  e.s0 = lo < gamma ? sin_tab[lo] : inf;
  e.s1 = lo + 1 < gamma ? sin_tab[lo + 1] : inf;
  e.s2 = lo + 2 < gamma ? sin_tab[lo + 2] : inf;
  bins[b] = e;
}

// ------------------------------------------------------------------ input checks
__global__ void validate_kernel(const float* __restrict__ xyz, uint32_t nv,
                                const uint32_t* __restrict__ idx, uint64_t nidx,
                                uint32_t* __restrict__ bad) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 3ull * nv && !isfinite(xyz[i])) atomicOr(bad, 1u);
  if (idx && i < nidx && idx[i] >= nv) atomicOr(bad, 2u);
}

__global__ void pad_kernel(const float* __restrict__ xyz, uint32_t nv, float4* __restrict__ v) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  v[i] = make_float4(xyz[3ull * i], xyz[3ull * i + 1], xyz[3ull * i + 2], 0.0f);
}

__global__ void split_kernel(const float4* __restrict__ v, uint32_t n, float* __restrict__ x,
                             float* __restrict__ y, float* __restrict__ z) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 p = v[i];
  x[i] = p.x;
  y[i] = p.y;
  z[i] = p.z;
}

// ================================================================== launchers
static inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

hipError_t launch_init(unsigned long long* keys, uint32_t n, Counters* cnt, hipStream_t st) {
  constexpr uint32_t WORDS = (uint32_t)(sizeof(Counters) / sizeof(uint32_t));
  const uint32_t nb = cdiv(n > WORDS ? n : WORDS, 256);
  hipLaunchKernelGGL(init_kernel, dim3(nb), dim3(256), 0, st, keys, n, cnt);
  return hipGetLastError();
}

hipError_t launch_bounds(const DevScene* scenes, uint32_t nscenes, uint32_t total_tiles,
                         uint32_t block, const DevSensor* sens, uint32_t small_c, uint32_t small_r,
                         Item* items, uint32_t* item_cs, uint32_t item_scap, Item* large,
                         uint32_t large_scap, Counters* cnt, uint32_t group_cull,
                         uint32_t inline_max, bool lossy, unsigned long long* keys,
                         hipStream_t st) {
  if (total_tiles == 0) return hipSuccess;
#define GRCA_BOUNDS_CASE(B)                                                                   \
  case B: {                                                                                   \
    constexpr uint32_t W = B / 64;                                                            \
    const uint32_t nb = cdiv(total_tiles, W);                                                 \
    if (lossy) {                                                                              \
      hipLaunchKernelGGL((bounds_kernel<W, false, true>), dim3(nb), dim3(B), 0, st, scenes,    \
                         nscenes, total_tiles, sens, small_c, small_r, items, item_cs,         \
                         item_scap, large, large_scap, cnt, group_cull, 0u, keys);             \
    } else if (inline_max) {                                                                  \
      hipLaunchKernelGGL((bounds_kernel<W, true, false>), dim3(nb), dim3(B), 0, st, scenes,    \
                         nscenes, total_tiles, sens, small_c, small_r, items, item_cs,         \
                         item_scap, large, large_scap, cnt, group_cull, inline_max, keys);     \
    } else {                                                                                  \
      hipLaunchKernelGGL((bounds_kernel<W, false, false>), dim3(nb), dim3(B), 0, st, scenes,   \
                         nscenes, total_tiles, sens, small_c, small_r, items, item_cs,         \
                         item_scap, large, large_scap, cnt, group_cull, 0u, keys);             \
    }                                                                                         \
    break;                                                                                    \
  }
  switch (block) {
    GRCA_BOUNDS_CASE(64)
    GRCA_BOUNDS_CASE(128)
    GRCA_BOUNDS_CASE(256)
    GRCA_BOUNDS_CASE(512)
    GRCA_BOUNDS_CASE(1024)
    default:
      return hipErrorInvalidValue;
  }
#undef GRCA_BOUNDS_CASE
  return hipGetLastError();
}

hipError_t launch_expand(const DevScene* scenes, const DevSensor* sens, const Item* large,
                         Item* items, uint32_t* item_cs, uint32_t item_scap, uint32_t large_scap,
                         uint32_t row_chunk, Counters* cnt, uint32_t nblocks, hipStream_t st) {
  hipLaunchKernelGGL(expand_kernel<4>, dim3(nblocks), dim3(256), 0, st, scenes, sens, large,
                     items, item_cs, item_scap, large_scap, row_chunk, cnt);
  return hipGetLastError();
}

hipError_t launch_isect(const DevScene* scenes, const DevSensor* sens, uint32_t nsens,
                        const Item* items, const uint32_t* item_cs, uint32_t item_scap,
                        uint32_t ticket_cands, Counters* cnt, unsigned long long* keys,
                        uint32_t nblocks, hipStream_t st) {
  if (nsens <= 64)
    hipLaunchKernelGGL((isect_kernel<4, true>), dim3(nblocks), dim3(256), 0, st, scenes, sens,
                       nsens, items, item_cs, item_scap, ticket_cands, cnt, keys);
  else
    hipLaunchKernelGGL((isect_kernel<4, false>), dim3(nblocks), dim3(256), 0, st, scenes, sens,
                       nsens, items, item_cs, item_scap, ticket_cands, cnt, keys);
  return hipGetLastError();
}

hipError_t launch_allpairs(const DevScene* scenes, const DevSensor* sens, uint32_t sensor,
                           uint32_t ntri, uint32_t nrays, Statics* statics,
                           unsigned long long* keys, hipStream_t st) {
  if (ntri == 0 || nrays == 0) return hipSuccess;
  hipLaunchKernelGGL(statics_kernel, dim3(cdiv(ntri, 256)), dim3(256), 0, st, scenes, sens,
                     sensor, statics);
  const uint32_t chunk = 4096;
  hipLaunchKernelGGL(allpairs_kernel, dim3(cdiv(nrays, 256), cdiv(ntri, chunk)), dim3(256), 0,
                     st, sens, sensor, statics, ntri, chunk, keys);
  return hipGetLastError();
}

hipError_t launch_resolve(const unsigned long long* keys, uint32_t n, float* dist, uint32_t* tri,
                          Counters* cnt, hipStream_t st) {
  // 16-byte stores need 16-byte aligned outputs (caller buffers may be offset)
  const bool vec = (reinterpret_cast<uintptr_t>(dist) % 16u == 0) &&
                   (reinterpret_cast<uintptr_t>(tri) % 16u == 0);
  const uint32_t nb = cdiv(std::max(cdiv(n, 4u), 64u), 256u);
  if (vec)
    hipLaunchKernelGGL(resolve_kernel<true>, dim3(nb), dim3(256), 0, st, keys, n, dist, tri, cnt);
  else
    hipLaunchKernelGGL(resolve_kernel<false>, dim3(nb), dim3(256), 0, st, keys, n, dist, tri,
                       cnt);
  return hipGetLastError();
}

hipError_t launch_pose(const PoseBlock* rblocks, uint32_t n_rigid, const float* rrx,
                       const float* rry, const float* rrz, const PoseBlock* dblocks,
                       uint32_t n_deform, const float* drx, const float* dry, const float* drz,
                       const float* nx, const float* ny, const float* nz, const float* phase,
                       const DeformParam* groups, const double* pose_in, float4* v,
                       hipStream_t st) {
  if (n_rigid + n_deform == 0) return hipSuccess;
  hipLaunchKernelGGL(pose_kernel, dim3(n_rigid + n_deform), dim3(256), 0, st, rblocks, n_rigid,
                     rrx, rry, rrz, dblocks, drx, dry, drz, nx, ny, nz, phase, groups, pose_in, v);
  return hipGetLastError();
}

hipError_t launch_sensor_tables(const float* elev, const float* el_off, uint32_t gamma,
                                uint32_t chi, double dtheta, const float* az_off, float2* chan,
                                double2* chan_d, float* sin_tab, float2* az, uint32_t lut_size,
                                ChanBin* lut, hipStream_t st) {
  const uint32_t n = gamma > chi ? gamma : chi;
  hipLaunchKernelGGL(sensor_tables_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, elev, el_off,
                     gamma, chi, dtheta, az_off, chan, chan_d, sin_tab, az);
  hipLaunchKernelGGL(sensor_lut_kernel, dim3(cdiv(lut_size, 256)), dim3(256), 0, st, sin_tab,
                     gamma, lut_size, lut);
  return hipGetLastError();
}

hipError_t launch_validate(const float* xyz, uint32_t nv, const uint32_t* idx, uint64_t nidx,
                           uint32_t* bad, hipStream_t st) {
  const uint64_t n = 3ull * nv > nidx ? 3ull * nv : nidx;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(validate_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, xyz, nv, idx, nidx,
                     bad);
  return hipGetLastError();
}

hipError_t launch_spheres(const float4* soup, uint32_t n_pre, float4* tsph, float4* gsph,
                          hipStream_t st) {
  if (n_pre == 0) return hipSuccess;
  hipLaunchKernelGGL(sphere_kernel, dim3(cdiv(n_pre, 4)), dim3(256), 0, st, soup, n_pre, tsph,
                     gsph);
  return hipGetLastError();
}

hipError_t launch_pad(const float* xyz, uint32_t nv, float4* v, hipStream_t st) {
  if (nv == 0) return hipSuccess;
  hipLaunchKernelGGL(pad_kernel, dim3(cdiv(nv, 256)), dim3(256), 0, st, xyz, nv, v);
  return hipGetLastError();
}

hipError_t launch_split(const float4* v, uint32_t n, float* x, float* y, float* z,
                        hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(split_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, v, n, x, y, z);
  return hipGetLastError();
}

// ------------------------------------------------------ no-allocation casts
// Work memory of the no-allocation cast: counters, the cast's sensor and
// scene descriptors, the keys and the work queues, carved by the host from
// this one array.  Each device the library runs on holds its own copy for
// the life of the process.  Host code must not pass the array's name to a
// kernel (on the host it names a stand-in, not device memory): it uses the
// device address that noalloc_scratch_address returns.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch_address(void** out) {
  return hipGetSymbolAddress(out, HIP_SYMBOL(scratch));
}

// Copies a small host record into device memory through the kernel's
// arguments: nothing is staged in host memory that a later call could
// overwrite before the copy runs, and nothing is allocated.
struct PutBlob {
  uint32_t words;
  uint32_t w[PUT_BLOB_WORDS];
};
static_assert(sizeof(PutBlob) <= 4096, "kernel arguments are limited to 4 KiB");

__global__ void put_kernel(uint32_t* __restrict__ dst, PutBlob b) {
  for (uint32_t i = threadIdx.x; i < b.words; i += blockDim.x) dst[i] = b.w[i];
}

hipError_t launch_put(void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (bytes % 4u != 0u || reinterpret_cast<uintptr_t>(dst) % 4u != 0u) return hipErrorInvalidValue;
  const uint32_t* s = static_cast<const uint32_t*>(src);
  uint32_t* d = static_cast<uint32_t*>(dst);
  size_t left = bytes / 4u;
  while (left) {
    PutBlob b;
    b.words = (uint32_t)std::min<size_t>(left, PUT_BLOB_WORDS);
    for (uint32_t i = 0; i < b.words; ++i) b.w[i] = s[i];
    hipLaunchKernelGGL(put_kernel, dim3(1), dim3(256), 0, st, d, b);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    s += b.words;
    d += b.words;
    left -= b.words;
  }
  return hipSuccess;
}

}  // namespace grca

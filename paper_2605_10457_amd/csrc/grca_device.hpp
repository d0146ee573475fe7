// grca_device.hpp -- device-side data layout and per-pair arithmetic shared by
// every kernel of the caster (bounds/binning, large-class expansion,
// cooperative intersection, all-pairs reference).
//
// All paths evaluate a (ray, triangle) pair with the same two functions
// (make_statics + ray_test), so the culled cast and the all-pairs reference
// are bitwise comparable.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace grca {

// (f_sort(+inf) << 32) | miss id: the initial key of every ray.  f_sort is the
// order-preserving float -> uint32 map of appendix "Per-Ray Distance
// Encoding"; the low word carries the triangle id so that a 64-bit minimum
// selects the closest hit and, at equal FP32 distance, the smaller id.
constexpr unsigned long long KEY_INIT = 0xFF800000FFFFFFFFull;
constexpr uint32_t MISS = 0xFFFFFFFFu;

// Work-item record (16 B).  A rectangle of candidate rays of one
// (triangle, sensor) pair: channels [c_from, c_from + c_count) x rays
// [r_start, r_start + r_count) (ray index mod chi on full-spin sensors).
// Large-class records use the same layout with r_count = 0 (rays are
// computed per channel by the expansion kernel).
struct Item {
  uint32_t tri;
  uint32_t chan;   // c_from | c_count << 16
  uint32_t rays;   // r_start | r_count << 16
  uint32_t sensor; // sensor slot of the cast
};

// One bin of the sine -> channel lookup: the first channel j whose sine is
// >= the bin's lower edge -1 + 2b/lut_size, and the sines of channels j, j+1,
// j+2 (+inf past the last channel), so that a search usually needs one load.
struct ChanBin {
  uint32_t j;
  float s0, s1, s2;
};

// Per-cast sensor descriptor (device memory; read with wave-uniform indices,
// except in the span phase of the bounds pass, where each lane reads its own).
struct alignas(16) DevSensor {
  float o[3], f[3], r[3], u[3];
  float dmin, dmax;
  // max |elevation offset| (radians), widens every channel span; the paper's
  // lossy accelerations enabled for this cast (GRCA_LOSSY_* bits, 0 in an
  // exact cast).  Next to the range, so the span reads them in one load.
  float el_noise;
  uint32_t lossy;
  uint32_t gamma, chi;
  uint32_t key_offset; // O_n: first output slot of this sensor
  uint32_t wrap;       // 1: full spin, azimuth index wraps mod chi
  uint32_t scene;      // scene slot of the cast
  uint32_t lut_size;   // bins of the sine -> channel lookup
  float theta_start;   // theta_0 = -floor(chi/2) * dtheta (FP32 copy for the bounds pass)
  float inv_dtheta;    // chi / fov
  float period_idx;    // 2 pi / dtheta: one full turn in ray-index units
  int32_t cull_back;   // 0: two-sided; +1/-1: single-sided, sign = handedness of (f, r, u)
  double theta_start_d, inv_dtheta_d, period_idx_d;
  const float2* chan;   // (cos phi_j, sin phi_j), FP32
  const double2* chan_d; // (cos phi_j, sin phi_j), FP64
  const float* sin_tab; // sin phi_j of the nominal table (FP32), ascending (chan and
                        // chan_d hold the perturbed elevations under vertical noise)
  const ChanBin* bins;  // lut_size bins of the sine -> channel lookup
  const float2* az;     // (cos theta_R, sin theta_R), FP32 (offsets included)
  const uint8_t* mask;  // optional active-ray mask at C * chi + R (nullptr: all on)
  float az_noise;       // max |azimuth offset| (radians), widens every azimuth span
  // the channel elevations as a uniform grid, for the first test of the
  // bounds pass: every channel j lies within elev_tol of elev0 + j / inv_delev
  float elev0, inv_delev, elev_tol;
  // the sphere tests' per-sensor constants: range thresholds with their
  // margins (cull beyond dmax (1 + 1e-5) + 1e-6; wholly inside
  // (dmin (1 + 1e-5), dmax (1 - 1e-5))), the elevation margin 3e-5 +
  // elev_tol, the last channel index gamma - 1 and elev0 * inv_delev
  float cull_dmax, in_dmax, in_dmin, elev_m, last_chan, elev0_g;
  float eps_area;  // the apparent-area threshold epsilon_A of GRCA_LOSSY_AREA
  // a partial field of view as the wedge between two vertical planes through
  // the origin, for the sphere tests: fov_mode 0 = no test (full spin, or a
  // wedge that the margins widen to a full turn), 1 = the wedge is convex
  // (at most pi wide: the intersection of the planes' inner half-spaces),
  // 2 = wider (their union); fov_n = the inward unit normals (f and r
  // components) of the start and end planes, each turned outward by 1e-4 rad
  // plus the azimuth noise
  uint32_t fov_mode;
  float fov_n[4];
  // 1: the up axis is the world z axis within 1e-4 (|u_x| + |u_y|), so that
  // the triangle tests may bound a triangle by an upright cylinder
  uint32_t upright;
  uint32_t pad_[3];
};

static_assert(sizeof(DevSensor) % 16 == 0 && offsetof(DevSensor, dmin) % 16 == 0 &&
                  offsetof(DevSensor, lossy) ==
                  offsetof(DevSensor, dmin) + 12,
              "range, vertical noise and lossy bits form one aligned 16-byte block");

// Triangles per tile of the bounds pass: one wave, two triangles per lane.
constexpr uint32_t BOUNDS_TILE = 128;

struct DevScene {
  const float4* v;       // vertex positions (x, y, z, 0): one 16-byte load per vertex
  // the static triangles' vertex records, three per triangle (48 B), for
  // slots [0, n_soup): the tile order puts every triangle whose vertices are
  // all static first; no pose moves them, so these copies stay current.  The
  // intersection reads a static triangle here in one round trip instead of
  // its indices and then its vertices
  const float4* soup;
  // bounding spheres of the first n_pre tiles (all-static, full tiles),
  // computed at scene setup as the bounds pass would: per triangle (tsph,
  // 128 per tile) and per tile (gsph)
  const float4* tsph;
  const float4* gsph;
  uint32_t n_pre;
  const uint32_t* idx;   // index triples in tile order
  const uint32_t* orig;  // caller triangle id of each stored slot (keys and outputs use it)
  uint32_t ntri;
  uint32_t n_soup;       // slots with a vertex record copy in `soup`
  uint32_t tile_start;   // first bounds tile (BOUNDS_TILE triangles) of this scene in the cast
  uint32_t sensor_begin; // sensor slots [sensor_begin, sensor_end) observe it
  uint32_t sensor_end;
};

// Work queues are split into NSHARD equal regions, each with its own append
// counter and consumer ticket on a cache line of its own.  Atomics that many
// waves aim at one address are serialised by the memory system (about 11 ns
// apiece on gfx950, measured), so a producer wave appends to, and a consumer
// wave takes tickets from, the shard of its own global wave index only.
constexpr uint32_t NSHARD = 64;

struct alignas(256) Shard {
  // Item shards: reserved slots in the low word (may exceed the shard's
  // capacity: overflow) and reserved candidate pairs in the high word, so one
  // 64-bit atomic keeps both in the same order.  Large-record shards use the
  // low word only.
  unsigned long long nc;
  uint32_t tk;              // tickets handed out by the intersection (item shards)
  uint32_t rows;            // row items appended by the expansion (statistic)
  unsigned long long rtic;  // candidate pairs executed from this shard (statistic)
  unsigned long long pairs; // (triangle, origin) spans computed (statistic)
  unsigned long long tests; // (triangle, origin) bounding-sphere tests (statistic)
  unsigned long long atomics; // 64-bit atomic minima issued on keys (statistic)
  uint32_t pad[52];
};
static_assert(sizeof(Shard) == 256, "one shard counter per 256-byte line");

// Overflow record that outlives a cast: the init kernel leaves it alone, so
// it accumulates over every cast run on the same counters (the launches of a
// frame) until the host clears it.
struct Sticky {
  uint32_t overflow;         // OR of the overflow bits of those casts
  uint32_t casts;            // how many of them overflowed
  uint32_t max_items_shard;  // largest item-shard request among them
  uint32_t max_large_shard;  // largest large-shard request among them
};

// Compact per-cast summary written at the end of a cast and copied to the host.
struct Summary {
  uint32_t n_items;          // item slots requested over all shards
  uint32_t n_large;          // large-class records requested
  uint32_t n_rows;           // of n_items: row items of the expansion
  uint32_t overflow;         // bit 0: item queue, bit 1: large queue, bit 2: candidate space
  uint32_t max_items_shard;  // largest request of one item shard
  uint32_t max_large_shard;  // largest request of one large-record shard
  unsigned long long rtic;   // candidate pairs executed
  unsigned long long pairs;  // (triangle, origin) spans computed
  unsigned long long tests;  // (triangle, origin) bounding-sphere tests
  unsigned long long atomics; // 64-bit atomic minima issued on keys
  Sticky sticky;             // the sticky record as this cast left it
};

// Device counters of one cast, cleared by the init kernel up to `sticky`.
struct Counters {
  Shard items[NSHARD];
  Shard large[NSHARD];
  alignas(256) uint32_t overflow;
  alignas(256) Summary sum;
  alignas(256) Sticky sticky;  // not cleared per cast (see Sticky)
};

// Per-(triangle, origin) statics of the ray test, all in the sensor's local
// frame (x = forward, y = right, z = up): unit normals of the three planes
// through the origin and each edge, oriented so the triangle's forward cone
// is their positive side; the unit face normal oriented away from the
// origin; and the origin-to-plane distance h.  With d the unit ray and
// w_k = d . n_k, Moller-Trumbore's barycentrics are (w_2, w_0, w_1) / (d . N)
// and its distance is h / (d . N_hat): the test below is the MT test with
// every ray-independent product precomputed once per pair.
struct Statics {
  float n0x, n0y, n0z, n1x;
  float n1y, n1z, n2x, n2y;
  float n2z, Nx, Ny, Nz;
  float h, pad0, pad1, pad2;
};

// `s` is any sensor record with the frame o, f, r, u and cull_back (the
// device descriptor, or its copy in LDS).
template <class SensorT>
__device__ inline bool make_statics(float ax, float ay, float az_, float bx, float by, float bz,
                                    float cx, float cy, float cz, const SensorT& s,
                                    Statics& st, double (*nrm_out)[3] = nullptr) {
  // FP64 throughout, rounded once to FP32 at the end.
  const double ox = s.o[0], oy = s.o[1], oz = s.o[2];
  const double fx = s.f[0], fy = s.f[1], fz = s.f[2];
  const double rx = s.r[0], ry = s.r[1], rz = s.r[2];
  const double ux = s.u[0], uy = s.u[1], uz = s.u[2];
  double P[3][3];
  const double wx[3] = {(double)ax - ox, (double)bx - ox, (double)cx - ox};
  const double wy[3] = {(double)ay - oy, (double)by - oy, (double)cy - oy};
  const double wz[3] = {(double)az_ - oz, (double)bz - oz, (double)cz - oz};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    P[k][0] = wx[k] * fx + wy[k] * fy + wz[k] * fz;
    P[k][1] = wx[k] * rx + wy[k] * ry + wz[k] * rz;
    P[k][2] = wx[k] * ux + wy[k] * uy + wz[k] * uz;
  }
  const double e1[3] = {P[1][0] - P[0][0], P[1][1] - P[0][1], P[1][2] - P[0][2]};
  const double e2[3] = {P[2][0] - P[0][0], P[2][1] - P[0][1], P[2][2] - P[0][2]};
  const double N[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                       e1[0] * e2[1] - e1[1] * e2[0]};
  const double g = P[0][0] * N[0] + P[0][1] * N[1] + P[0][2] * N[2];
  const double nN2 = N[0] * N[0] + N[1] * N[1] + N[2] * N[2];
  if (!(nN2 > 0.0) || g == 0.0 || !(g == g)) return false;
  const double sg = g > 0.0 ? 1.0 : -1.0;
  // Single-sided casting keeps only front faces, d . (e1 x e2) < 0 in world
  // coordinates; a hit has sign(d . N) = sign(p0 . N), and the local frame
  // flips that sign when (f, r, u) is left-handed.
  if (s.cull_back != 0 && (double)s.cull_back * sg > 0.0) return false;
  double n[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int k1 = (k + 1) % 3;
    const double E[3] = {P[k1][0] - P[k][0], P[k1][1] - P[k][1], P[k1][2] - P[k][2]};
    const double c0 = P[k][1] * E[2] - P[k][2] * E[1];
    const double c1 = P[k][2] * E[0] - P[k][0] * E[2];
    const double c2 = P[k][0] * E[1] - P[k][1] * E[0];
    const double l2 = c0 * c0 + c1 * c1 + c2 * c2;
    if (!(l2 > 0.0)) return false;
    const double il = sg * rsqrt(l2);
    n[k][0] = c0 * il;
    n[k][1] = c1 * il;
    n[k][2] = c2 * il;
  }
  const double iN = sg * rsqrt(nN2);
  st.n0x = (float)n[0][0]; st.n0y = (float)n[0][1]; st.n0z = (float)n[0][2];
  st.n1x = (float)n[1][0]; st.n1y = (float)n[1][1]; st.n1z = (float)n[1][2];
  st.n2x = (float)n[2][0]; st.n2y = (float)n[2][1]; st.n2z = (float)n[2][2];
  st.Nx = (float)(N[0] * iN); st.Ny = (float)(N[1] * iN); st.Nz = (float)(N[2] * iN);
  st.h = (float)(g * iN);
  st.pad0 = st.pad1 = st.pad2 = 0.0f;
  if (nrm_out) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      nrm_out[k][0] = n[k][0];
      nrm_out[k][1] = n[k][1];
      nrm_out[k][2] = n[k][2];
    }
  }
  return true;
}

// FP32 ray test with fixed evaluation order (no contraction beyond the
// explicit fmaf calls), so every call site rounds identically.
// Returns the packed key of a hit, or KEY_INIT.
__device__ inline unsigned long long ray_test(const Statics& st, float cphi, float sphi,
                                              float cth, float sth, float dmin, float dmax,
                                              uint32_t tri) {
#pragma clang fp contract(off)
  const float dx = cphi * cth;
  const float dy = cphi * sth;
  const float dz = sphi;
  const float w0 = fmaf(st.n0x, dx, fmaf(st.n0y, dy, st.n0z * dz));
  const float w1 = fmaf(st.n1x, dx, fmaf(st.n1y, dy, st.n1z * dz));
  const float w2 = fmaf(st.n2x, dx, fmaf(st.n2y, dy, st.n2z * dz));
  const float c = fmaf(st.Nx, dx, fmaf(st.Ny, dy, st.Nz * dz));
  // (the statics of a valid pair are finite, so the minimum of the three
  // barycentric numerators is a plain comparison)
  if (fminf(fminf(w0, w1), w2) >= 0.0f && c > 0.0f) {
    // hardware reciprocal (1 ulp) and one rounded product: t within 2 ulps
    // of h / c, the same at every call site
    const float t = st.h * __builtin_amdgcn_rcpf(c);
    if (t >= dmin && t <= dmax) {
      // f_sort(t) for t > 0 sets the sign bit; the miss key stays larger.
      const uint32_t u = __float_as_uint(t);
      const uint32_t m = (uint32_t)(-(int32_t)(u >> 31)) | 0x80000000u;
      return ((unsigned long long)(u ^ m) << 32) | (unsigned long long)tri;
    }
  }
  return KEY_INIT;
}

__device__ inline void key_min(unsigned long long* keys, uint32_t g, unsigned long long key) {
  atomicMin(keys + g, key);
}

}  // namespace grca

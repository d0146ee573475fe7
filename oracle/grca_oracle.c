/*
 * grca_oracle.c -- FP64 brute-force reference for emitter-centric closest-hit
 * LiDAR ray casting.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg may load this library.  It shares no
 * source, header, table or helper with the HIP implementation, and nothing in
 * the product path may call it.
 *
 * What it computes (the plain definition of the problem, section 1.1
 * "Problem Statement"): for every ray of every LiDAR, the closest triangle it
 * intersects and the distance to it.  There is no culling of any kind: every
 * ray is tested against every triangle.
 *
 *   - Ray directions follow section 3.1, Eq. (ray_dir):
 *       d = cos(theta) cos(phi) f + sin(theta) cos(phi) r + sin(phi) u,
 *     with the azimuth grid theta_R = (R - floor(chi/2)) * dtheta (section 3.1,
 *     centred start offset) generalised to a partial field of view,
 *     dtheta = fov / chi, and the elevation phi_C taken from an explicit
 *     ascending per-channel table (C = 0 is the lowest channel).
 *   - The ray-triangle test is two-sided Moller-Trumbore (the RTIC named in
 *     appendix "Two Pass Pipeline Detail", early pass step 5), evaluated in
 *     FP64 on the FP32 inputs promoted exactly to FP64.
 *   - A hit counts iff the barycentrics are inside (bounds inclusive) and the
 *     distance lies in [range_min, range_max] (the range limits of the
 *     origin-centric filters, appendix early pass step 1, applied per hit).
 *   - The closest hit is the lexicographic minimum of (t, triangle id), the
 *     order that the sortable distance encoding of appendix "Per-Ray Distance
 *     Encoding" extended by the triangle id produces.
 *
 * Beyond the hit itself, every ray gets flags that mark where FP32 and FP64
 * may legitimately disagree (grazing edges, near ties, range edges, grazing
 * incidence).  These are reporting aids for the parity tests; they do not
 * change the hit.
 *
 * The pose step (rigid instance transforms and per-vertex sinusoidal
 * deformation of the dynamic geometry) is the plain formula evaluated in FP64
 * and rounded once to FP32, the precision of the scene's vertex buffer.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- flags --------------------------------------------------------------- */
#define ORC_GRAZING            1u  /* ray within GRAZE_RAD of a relevant triangle's boundary */
#define ORC_NEAR_TIE           2u  /* best and second-best triangles within the band in t    */
#define ORC_RANGE_EDGE         4u  /* a hit within the band of range_min or range_max that is
                                      not behind the closest in-range hit                   */
#define ORC_GRAZING_INCIDENCE  8u  /* |d . n| of the hit triangle below INCIDENCE_COS         */

#define GRAZE_RAD     1e-6
#define TIE_REL       1e-5
#define INCIDENCE_COS 0.05

/* Relative half-width of the band within which a single-precision evaluation
 * of a hit distance may legitimately differ from this FP64 one: TIE_REL, the
 * distance tolerance of the parity criterion, widened in proportion to
 * 1/|cos| below INCIDENCE_COS, because t = h / (d . n) amplifies the absolute
 * error of the direction by 1/|cos incidence|.  Two distances whose bands
 * overlap may come out in either order; a distance whose band contains a
 * range limit may fall on either side of it. */
static double dist_band(double cos_abs) {
  if (cos_abs >= INCIDENCE_COS) return TIE_REL;
  return TIE_REL * INCIDENCE_COS / (cos_abs > 1e-300 ? cos_abs : 1e-300);
}

typedef struct {
  float origin[3];
  float forward[3];
  float right[3];
  float up[3];
  uint32_t num_channels;
  uint32_t rays_per_channel;
  const float* channel_elevation_rad;
  float fov_rad;
  float range_min;
  float range_max;
  uint32_t flags; /* bit 0: single-sided (cull back faces) */
  const float* azimuth_offset_rad; /* optional, chi values: theta*_R = theta_R + offset_R */
  const uint8_t* ray_mask;         /* optional, gamma*chi values: 0 = ray switched off  */
  const float* channel_elevation_offset_rad; /* optional, gamma values: phi*_C = phi_C +
                                                offset_C (per-channel vertical noise)     */
} oracle_sensor;

/* ---- small vector helpers (FP64) ---------------------------------------- */
static void sub3(const double* a, const double* b, double* o) {
  o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2];
}
static double dot3(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void cross3(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double* a) { return sqrt(dot3(a, a)); }

static void load_vertex(const float* xyz, uint32_t i, double* o) {
  o[0] = (double)xyz[3 * (size_t)i + 0];
  o[1] = (double)xyz[3 * (size_t)i + 1];
  o[2] = (double)xyz[3 * (size_t)i + 2];
}

/* Ray direction of channel C, ray R (section 3.1, Eq. ray_dir), normalised. */
void oracle_ray_direction(const oracle_sensor* s, uint32_t C, uint32_t R, double* d) {
  const double chi = (double)s->rays_per_channel;
  const double dtheta = (double)s->fov_rad / chi;
  double theta = ((double)R - floor(chi / 2.0)) * dtheta;
  /* angular noise (appendix "Ray Noise Simulation"): a pre-stored perturbed azimuth */
  if (s->azimuth_offset_rad) theta += (double)s->azimuth_offset_rad[R];
  double phi = (double)s->channel_elevation_rad[C];
  /* per-channel vertical noise (same appendix): a pre-stored perturbed elevation */
  if (s->channel_elevation_offset_rad) phi += (double)s->channel_elevation_offset_rad[C];
  const double ct = cos(theta), st = sin(theta), cp = cos(phi), sp = sin(phi);
  for (int k = 0; k < 3; ++k)
    d[k] = ct * cp * (double)s->forward[k] + st * cp * (double)s->right[k] +
           sp * (double)s->up[k];
  const double n = norm3(d);
  d[0] /= n; d[1] /= n; d[2] /= n;
}

/* Two-sided Moller-Trumbore (1997) in FP64.  Returns 1 when the ray meets the
 * triangle's face (barycentrics inside, inclusive) at parameter *t; the range
 * check is left to the caller.  det == 0 (ray parallel to the plane, or a
 * degenerate triangle) is a miss. */
static int mt_fp64(const double* o, const double* d, const double* a, const double* b,
                   const double* c, int single_sided, double* t, double* det_out) {
  double e1[3], e2[3], p[3], s[3], q[3];
  sub3(b, a, e1);
  sub3(c, a, e2);
  cross3(d, e2, p);
  const double det = dot3(e1, p);
  *det_out = det;
  if (det == 0.0) return 0;
  if (single_sided && !(det > 0.0)) return 0; /* front face: d . (e1 x e2) < 0 */
  const double inv = 1.0 / det;
  sub3(o, a, s);
  const double u = dot3(s, p) * inv;
  cross3(s, e1, q);
  const double v = dot3(d, q) * inv;
  *t = dot3(e2, q) * inv;
  return (u >= 0.0 && v >= 0.0 && u + v <= 1.0);
}

/* Signed angular margins of direction d against the three planes through o
 * and each edge, oriented so that the triangle's forward cone is positive.
 * m[k] = d . n_k with n_k the unit normal of plane (o, v_k, v_{k+1}).  The
 * ray is inside the triangle's cone iff all m[k] >= 0; min m[k] is the sine
 * of its angle to the nearest edge plane.  Returns 0 if the triangle is
 * degenerate as seen from o (origin in its plane or zero area). */
static int edge_margins(const double* o, const double* d, const double* v0, const double* v1,
                        const double* v2, double* m, double* plane_t, double* cos_inc) {
  double p[3][3], n[3], N[3], e1[3], e2[3];
  sub3(v0, o, p[0]);
  sub3(v1, o, p[1]);
  sub3(v2, o, p[2]);
  sub3(v1, v0, e1);
  sub3(v2, v0, e2);
  cross3(e1, e2, N);
  const double nN = norm3(N);
  const double g = dot3(p[0], N); /* triple product p0 . (p1 x p2) */
  if (nN == 0.0 || g == 0.0) return 0;
  const double sg = g > 0.0 ? 1.0 : -1.0;
  for (int k = 0; k < 3; ++k) {
    cross3(p[k], p[(k + 1) % 3], n);
    const double nn = norm3(n);
    m[k] = nn > 0.0 ? sg * dot3(d, n) / nn : 0.0;
  }
  const double dn = dot3(d, N) / nN; /* cosine of incidence, signed */
  *cos_inc = dn;
  *plane_t = (dn != 0.0) ? (g / nN) / dn : INFINITY;
  return 1;
}

/* ---- per-ray brute force -------------------------------------------------- */
typedef struct {
  const oracle_sensor* s;
  const float* xyz;
  const uint32_t* idx;
  uint64_t ntri;
  const uint32_t* rays; /* global ray ids g = C * chi + R within this sensor */
  uint64_t nrays;
  double* out_t;
  uint32_t* out_tri;
  uint32_t* out_flags;
  double* out_t2;
  uint32_t* out_tri2;
  uint64_t next; /* work counter, guarded by mu */
  pthread_mutex_t mu;
} cast_job;

static void cast_one(const cast_job* J, uint64_t i) {
  const oracle_sensor* s = J->s;
  const uint32_t g = J->rays[i];
  const uint32_t chi = s->rays_per_channel;
  const uint32_t C = g / chi, R = g % chi;
  if (s->ray_mask && !s->ray_mask[g]) { /* switched-off ray (non-spinning patterns) */
    J->out_t[i] = INFINITY;
    J->out_tri[i] = 0xFFFFFFFFu;
    J->out_flags[i] = 0;
    if (J->out_t2) J->out_t2[i] = INFINITY;
    if (J->out_tri2) J->out_tri2[i] = 0xFFFFFFFFu;
    return;
  }
  double o[3] = {s->origin[0], s->origin[1], s->origin[2]};
  double d[3];
  oracle_ray_direction(s, C, R, d);
  const double dmin = (double)s->range_min, dmax = (double)s->range_max;
  const int single = (int)(s->flags & 1u);

  /* pass 1: closest hit = lexicographic min of (t, k); second best on another
   * triangle; the nearest face hit whose distance band holds a range limit */
  double t1 = INFINITY, t2 = INFINITY, b1 = TIE_REL, b2 = TIE_REL;
  double te = INFINITY, be = TIE_REL;
  uint32_t k1 = 0xFFFFFFFFu, k2 = 0xFFFFFFFFu;
  uint32_t flags = 0;
  for (uint64_t k = 0; k < J->ntri; ++k) {
    double a[3], b[3], c[3], t, det;
    load_vertex(J->xyz, J->idx[3 * k + 0], a);
    load_vertex(J->xyz, J->idx[3 * k + 1], b);
    load_vertex(J->xyz, J->idx[3 * k + 2], c);
    if (!mt_fp64(o, d, a, b, c, single, &t, &det)) continue;
    /* |cos incidence| = |det| / |e1 x e2| for a unit d (det = -d . (e1 x e2)) */
    double e1[3], e2[3], N[3];
    sub3(b, a, e1); sub3(c, a, e2); cross3(e1, e2, N);
    const double band = dist_band(fabs(det) / norm3(N));
    if ((fabs(t - dmin) <= band * dmin || fabs(t - dmax) <= band * dmax) && t < te) {
      te = t; be = band;
    }
    if (!(t >= dmin && t <= dmax)) continue;
    const uint32_t kk = (uint32_t)k;
    if (t < t1 || (t == t1 && kk < k1)) {
      t2 = t1; k2 = k1; b2 = b1;
      t1 = t; k1 = kk; b1 = band;
    } else if (t < t2 || (t == t2 && kk < k2)) {
      t2 = t; k2 = kk; b2 = band;
    }
  }
  if (k2 != 0xFFFFFFFFu && t2 - t1 <= fmax(b1, b2) * t1) flags |= ORC_NEAR_TIE;
  /* a range-edge hit matters only if it is not behind the closest in-range
   * hit (beyond their bands): a hidden one cannot change the answer */
  if (te < INFINITY && (k1 == 0xFFFFFFFFu || te <= t1 * (1.0 + fmax(b1, be))))
    flags |= ORC_RANGE_EDGE;

  /* pass 2: grazing -- a triangle whose angular boundary passes within
   * GRAZE_RAD of the ray and which is not hidden behind the best hit. */
  const double sg = sin(GRAZE_RAD);
  for (uint64_t k = 0; k < J->ntri; ++k) {
    double a[3], b[3], c[3], m[3], pt, ci;
    load_vertex(J->xyz, J->idx[3 * k + 0], a);
    load_vertex(J->xyz, J->idx[3 * k + 1], b);
    load_vertex(J->xyz, J->idx[3 * k + 2], c);
    int relevant;
    if (!edge_margins(o, d, a, b, c, m, &pt, &ci)) continue; /* never hit */
    const double mmin = fmin(m[0], fmin(m[1], m[2]));
    if (!(mmin >= -sg && mmin <= sg)) continue;
    /* depth relevance: plane distance, or vertex distances when seen edge-on */
    double pa[3], pb[3], pc[3];
    sub3(a, o, pa); sub3(b, o, pb); sub3(c, o, pc);
    const double ra = norm3(pa), rb = norm3(pb), rc = norm3(pc);
    const double rlo = fmin(ra, fmin(rb, rc)), rhi = fmax(ra, fmax(rb, rc));
    if (fabs(ci) * rlo <= sg * rhi || !isfinite(pt)) {
      relevant = rhi >= dmin * (1.0 - TIE_REL) && rlo <= dmax * (1.0 + TIE_REL) &&
                 (k1 == 0xFFFFFFFFu || rlo <= t1 * (1.0 + TIE_REL));
    } else {
      relevant = pt > 0.0 && pt >= dmin * (1.0 - TIE_REL) && pt <= dmax * (1.0 + TIE_REL) &&
                 (k1 == 0xFFFFFFFFu || pt <= t1 * (1.0 + TIE_REL));
    }
    if (relevant) { flags |= ORC_GRAZING; break; }
  }

  if (k1 != 0xFFFFFFFFu) {
    double a[3], b[3], c[3], e1[3], e2[3], N[3];
    load_vertex(J->xyz, J->idx[3 * (uint64_t)k1 + 0], a);
    load_vertex(J->xyz, J->idx[3 * (uint64_t)k1 + 1], b);
    load_vertex(J->xyz, J->idx[3 * (uint64_t)k1 + 2], c);
    sub3(b, a, e1); sub3(c, a, e2); cross3(e1, e2, N);
    if (fabs(dot3(d, N)) < INCIDENCE_COS * norm3(N)) flags |= ORC_GRAZING_INCIDENCE;
  }
  J->out_t[i] = t1;
  J->out_tri[i] = k1;
  J->out_flags[i] = flags;
  if (J->out_t2) J->out_t2[i] = t2;
  if (J->out_tri2) J->out_tri2[i] = k2;
}

static void* cast_worker(void* arg) {
  cast_job* J = (cast_job*)arg;
  const uint64_t chunk = 4;
  for (;;) {
    pthread_mutex_lock(&J->mu);
    const uint64_t b = J->next;
    J->next += chunk;
    pthread_mutex_unlock(&J->mu);
    if (b >= J->nrays) break;
    const uint64_t e = b + chunk < J->nrays ? b + chunk : J->nrays;
    for (uint64_t i = b; i < e; ++i) cast_one(J, i);
  }
  return NULL;
}

/* Cast the listed rays of one sensor against every triangle.
 * Outputs per listed ray: closest t (FP64, +inf on miss), triangle id
 * (0xFFFFFFFF on miss), flags, and the second-best (t, id) on another
 * triangle (optional, may be NULL).  Returns the number of threads used. */
int oracle_cast(const oracle_sensor* s, const float* xyz, const uint32_t* idx, uint64_t ntri,
                const uint32_t* rays, uint64_t nrays, int nthreads, double* out_t,
                uint32_t* out_tri, uint32_t* out_flags, double* out_t2, uint32_t* out_tri2) {
  cast_job J;
  memset(&J, 0, sizeof(J));
  J.s = s; J.xyz = xyz; J.idx = idx; J.ntri = ntri; J.rays = rays; J.nrays = nrays;
  J.out_t = out_t; J.out_tri = out_tri; J.out_flags = out_flags;
  J.out_t2 = out_t2; J.out_tri2 = out_tri2;
  pthread_mutex_init(&J.mu, NULL);
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  pthread_t th[256];
  for (int i = 0; i < nthreads; ++i) pthread_create(&th[i], NULL, cast_worker, &J);
  for (int i = 0; i < nthreads; ++i) pthread_join(th[i], NULL);
  pthread_mutex_destroy(&J.mu);
  return nthreads;
}

/* FP64 evaluation of one (ray, triangle) pair, for the parity checker.
 * out[0] = MT face hit (1/0, range ignored), out[1] = MT t, out[2] = min edge
 * margin (sine of angle to the nearest edge plane, negative outside),
 * out[3] = plane distance along the ray, out[4] = signed cos of incidence,
 * out[5] = 1 if the triangle is degenerate as seen from the origin. */
void oracle_pair(const oracle_sensor* s, const float* xyz, const uint32_t* idx, uint32_t g,
                 uint32_t k, double* out) {
  const uint32_t chi = s->rays_per_channel;
  double o[3] = {s->origin[0], s->origin[1], s->origin[2]};
  double d[3], a[3], b[3], c[3], t = NAN, det, m[3] = {0, 0, 0}, pt = NAN, ci = 0;
  oracle_ray_direction(s, g / chi, g % chi, d);
  load_vertex(xyz, idx[3 * (uint64_t)k + 0], a);
  load_vertex(xyz, idx[3 * (uint64_t)k + 1], b);
  load_vertex(xyz, idx[3 * (uint64_t)k + 2], c);
  const int hit = mt_fp64(o, d, a, b, c, (int)(s->flags & 1u), &t, &det);
  const int ok = edge_margins(o, d, a, b, c, m, &pt, &ci);
  out[0] = hit ? 1.0 : 0.0;
  out[1] = t;
  out[2] = ok ? fmin(m[0], fmin(m[1], m[2])) : 0.0;
  out[3] = pt;
  out[4] = ci;
  out[5] = ok ? 0.0 : 1.0;
}

/* ---- pose of the dynamic geometry ----------------------------------------- */

/* Rigid instance transform v' = M[:, 0:3] v + M[:, 3] for a vertex range,
 * M row-major 3x4 in FP32, evaluated in FP64 and rounded once to FP32. */
void oracle_pose_rigid(const float* rest_xyz, uint64_t n, const float* M, float* out_xyz) {
  for (uint64_t i = 0; i < n; ++i) {
    const double x = rest_xyz[3 * i], y = rest_xyz[3 * i + 1], z = rest_xyz[3 * i + 2];
    for (int r = 0; r < 3; ++r)
      out_xyz[3 * i + r] = (float)((double)M[4 * r] * x + (double)M[4 * r + 1] * y +
                                   (double)M[4 * r + 2] * z + (double)M[4 * r + 3]);
  }
}

/* Sinusoidal deformation v' = v + A sin(omega * time + phase_v) n_v, in FP64
 * (time in seconds, omega in rad/s), rounded once to FP32. */
void oracle_pose_deform(const float* rest_xyz, const float* normal_xyz, const float* phase,
                        uint64_t n, float amplitude, float omega, double time, float* out_xyz) {
  for (uint64_t i = 0; i < n; ++i) {
    const double w = (double)amplitude * sin((double)omega * time + (double)phase[i]);
    for (int r = 0; r < 3; ++r)
      out_xyz[3 * i + r] = (float)((double)rest_xyz[3 * i + r] + w * (double)normal_xyz[3 * i + r]);
  }
}

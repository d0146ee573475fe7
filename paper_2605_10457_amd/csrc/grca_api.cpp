// grca_api.cpp -- host runtime behind the C ABI of include/grca.h.
//
// Owns the device-resident scenes (16-byte vertex records + indices, the
// static triangles' record copies and spheres, rest geometry of dynamic
// ranges), the sensor tables, the per-cast workspaces (ray keys, work
// queues, counters) and the hipGraph frames.  Every step of a cast runs in
// the HIP kernels of grca_kernels.hip; this file validates inputs, sizes
// buffers, enqueues launches and handles queue overflow by growing and
// recasting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "grca.h"
#include "grca_launch.hpp"

using namespace grca;

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

struct SceneData {
  uint32_t nv = 0, ntri = 0;
  float4* v = nullptr;       // vertex positions (x, y, z, 0)
  float4* soup = nullptr;    // vertex records of the all-static triangles (slots [0, n_soup))
  uint32_t n_soup = 0;
  float4* tsph = nullptr;    // bounding spheres of the first n_pre tiles (triangles, tiles)
  float4* gsph = nullptr;
  uint32_t n_pre = 0;
  uint32_t* idx = nullptr;   // index triples in tile order (Morton within dynamic groups)
  uint32_t* orig = nullptr;  // caller triangle id of each stored slot
  // rigid instances
  uint32_t n_inst = 0;
  std::vector<uint32_t> inst_start, inst_count;
  float *rr_x = nullptr, *rr_y = nullptr, *rr_z = nullptr;  // rigid rest SoA
  PoseBlock* rigid_blocks = nullptr;
  uint32_t n_rigid_blocks = 0;
  // deform groups
  uint32_t n_groups = 0;
  std::vector<grca_deform_group> groups;
  float *dr_x = nullptr, *dr_y = nullptr, *dr_z = nullptr;  // deform rest SoA
  float *dn_x = nullptr, *dn_y = nullptr, *dn_z = nullptr, *dphase = nullptr;
  PoseBlock* deform_blocks = nullptr;
  uint32_t n_deform_blocks = 0;
  DeformParam* dparams = nullptr;
  // pose inputs: [time (double)][n_inst * 12 floats]
  double* pose_in = nullptr;
  unsigned char* pose_stage = nullptr;  // pinned
  size_t pose_bytes = 0;
  hipEvent_t pose_ev = nullptr;
};

struct SensorData {
  grca_sensor_desc desc{};
  std::vector<float> elev;
  float2* chan = nullptr;
  double2* chan_d = nullptr;
  float* sin_tab = nullptr;
  ChanBin* lut = nullptr;
  float2* az = nullptr;
  uint8_t* mask = nullptr;
  uint32_t lut_size = 0;
  float elev0 = 0.0f, inv_delev = 1.0f, elev_tol = 0.0f;  // channel grid (bounds pass)
  double dtheta = 0.0;
  float az_noise = 0.0f;
  float el_noise = 0.0f;  // max |channel elevation offset| (vertical noise), widened
  bool wrap = false;
};

template <typename T>
hipError_t dmalloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) return hipSuccess;
  return hipMalloc(reinterpret_cast<void**>(p), n * sizeof(T));
}
template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

void free_scene(SceneData& s) {
  dfree(s.v); dfree(s.soup); dfree(s.tsph); dfree(s.gsph); dfree(s.idx); dfree(s.orig);
  dfree(s.rr_x); dfree(s.rr_y); dfree(s.rr_z); dfree(s.rigid_blocks);
  dfree(s.dr_x); dfree(s.dr_y); dfree(s.dr_z);
  dfree(s.dn_x); dfree(s.dn_y); dfree(s.dn_z); dfree(s.dphase);
  dfree(s.deform_blocks); dfree(s.dparams); dfree(s.pose_in);
  if (s.pose_stage) (void)hipHostFree(s.pose_stage);
  s.pose_stage = nullptr;
  if (s.pose_ev) (void)hipEventDestroy(s.pose_ev);
  s.pose_ev = nullptr;
}

void free_sensor(SensorData& s) {
  dfree(s.chan); dfree(s.chan_d); dfree(s.sin_tab); dfree(s.lut); dfree(s.az); dfree(s.mask);
}

// Store the scene's triangles in tile order: Morton order of the centroids
// within each dynamic group (static geometry, each rigid instance, each
// deforming range), so that the bounds pass's tiles and their halves are compact
// and its tile-sphere test culls more.  `orig` keeps the caller's ids.
hipError_t reorder_scene_dev(SceneData& sc, hipStream_t st) {
  dfree(sc.soup);
  dfree(sc.tsph);
  dfree(sc.gsph);
  sc.soup = sc.tsph = sc.gsph = nullptr;
  sc.n_soup = sc.n_pre = 0;
  if (sc.ntri == 0 || sc.nv == 0) return hipSuccess;
  uint32_t* vg = nullptr;
  hipError_t e = dmalloc(&vg, sc.nv);
  if (e != hipSuccess) return e;
  e = launch_fill(vg, sc.nv, 0u, st);
  for (uint32_t i = 0; e == hipSuccess && i < sc.n_inst; ++i)
    e = launch_fill(vg + sc.inst_start[i], sc.inst_count[i], 1u + i, st);
  for (uint32_t g = 0; e == hipSuccess && g < sc.n_groups; ++g)
    e = launch_fill(vg + sc.groups[g].vertex_start, sc.groups[g].vertex_count,
                    1u + sc.n_inst + g, st);
  if (e == hipSuccess && sc.ntri >= 2)
    e = order_triangles(sc.idx, sc.orig, sc.ntri, sc.v, sc.nv, vg, st);
  uint32_t n_static = 0;
  if (e == hipSuccess) e = count_static(sc.idx, sc.ntri, vg, &n_static, st);
  (void)hipStreamSynchronize(st);
  dfree(vg);
  // the static triangles' vertex records (48 B each, addressed by 32-bit
  // byte offsets: at most 2^32 / 48 triangles get one)
  const uint32_t n_soup = std::min<uint32_t>(n_static, 0xFFFFFFFFu / 48u);
  if (e == hipSuccess && n_soup) {
    e = dmalloc(&sc.soup, 3ull * n_soup);
    if (e == hipSuccess) e = launch_soup(sc.idx, sc.v, n_soup, sc.soup, st);
    if (e == hipSuccess) sc.n_soup = n_soup;
  }
  // and the bounding spheres of the full tiles among them
  const uint32_t n_pre = sc.n_soup / BOUNDS_TILE;
  if (e == hipSuccess && n_pre) {
    e = dmalloc(&sc.tsph, (size_t)n_pre * BOUNDS_TILE);
    if (e == hipSuccess) e = dmalloc(&sc.gsph, n_pre);
    if (e == hipSuccess) e = launch_spheres(sc.soup, n_pre, sc.tsph, sc.gsph, st);
    if (e == hipSuccess) sc.n_pre = n_pre;
  }
  return e;
}

// Rewrite the static triangles' vertex records and spheres after their
// vertices changed.
hipError_t refresh_soup(SceneData& sc, hipStream_t st) {
  hipError_t e = launch_soup(sc.idx, sc.v, sc.n_soup, sc.soup, st);
  if (e == hipSuccess) e = launch_spheres(sc.soup, sc.n_pre, sc.tsph, sc.gsph, st);
  return e;
}

}  // namespace

constexpr int RING = 32;

struct CastRecord {
  bool live = false;
  std::vector<uint32_t> ids;
  float* dist = nullptr;
  uint32_t* tri = nullptr;
  uint32_t flags = 0;
  hipStream_t st = nullptr;
  uint64_t rays = 0, pairs = 0;
  uint32_t recasts = 0;
  uint32_t overflowed = 0;  // casts of this record whose queues overflowed
};

struct grca_workspace {
  grca_context* ctx = nullptr;
  unsigned long long* keys = nullptr;
  uint64_t key_cap = 0;
  Item* items = nullptr;
  uint32_t* item_cs = nullptr;    // first candidate index of each queued item (same capacity)
  uint64_t item_cap = 0;
  Item* large = nullptr;
  uint64_t large_cap = 0;
  Counters* cnt = nullptr;      // device counters (cleared by every cast's init kernel)
  Summary* cnt_host = nullptr;  // pinned, RING slots: each cast's summary
  hipEvent_t ev[RING] = {};
  CastRecord rec[RING];
  uint32_t next_slot = 0;
  int last_slot = -1;
  hipStream_t last_stream = nullptr;
  // per-slot staging of the cast's sensor / scene tables
  DevSensor* dsens = nullptr;        // device, RING * sens_cap
  DevSensor* dsens_host = nullptr;   // pinned, RING * sens_cap
  uint32_t sens_cap = 0;
  DevScene* dscenes = nullptr;
  DevScene* dscenes_host = nullptr;
  uint32_t scene_cap = 0;
  Statics* scratch = nullptr;
  uint64_t scratch_cap = 0;
  float* out_dist = nullptr;     // device staging for host outputs
  uint32_t* out_tri = nullptr;
  uint64_t out_cap = 0;
  bool fixed = false;            // capacity set by the user (serving)
  uint64_t bytes = 0;
};

struct grca_frame {
  grca_context* ctx = nullptr;
  uint32_t scene_id = 0;
  std::vector<uint32_t> ids;
  float* out_dist = nullptr;
  uint32_t* out_tri = nullptr;
  grca_workspace* ws = nullptr;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t tev[7] = {};  // stage events of grca_frame_profile
  bool stale = false;      // a scene or sensor it reads was reallocated: re-capture
  uint32_t lost = 0;       // overflowed launches not recast, not yet reported
};

constexpr uint32_t MAX_CAST_SENSORS = 4096;

// The plan of one cast: sensors grouped by scene, key offsets in caller order.
struct Plan {
  std::vector<DevSensor> sens;
  std::vector<DevScene> scenes;
  uint32_t total_tiles = 0;  // bounds tiles (BOUNDS_TILE triangles) over the cast's scenes
  uint64_t rays = 0;
  uint64_t pairs = 0;
};

struct grca_context {
  int device = 0;
  int num_cu = 0;
  std::map<uint32_t, SceneData> scenes;
  std::map<uint32_t, SensorData> sensors;
  grca_options opt{};
  grca_workspace* def_ws = nullptr;
  grca_workspace* last_ws = nullptr;
  std::set<grca_workspace*> workspaces;  // the default one and the caller's
  std::set<grca_frame*> frames;
  std::string err;
  // the planner's temporaries, reserved at creation for the largest cast
  // (4096 sensors), so that planning a cast never allocates
  std::vector<const SensorData*> plan_sd;
  std::vector<uint64_t> plan_off;
  std::vector<uint32_t> plan_order;
  // no-allocation casts: the device address of this device's static scratch
  // array, the plan (reserved for GRCA_NOALLOC_MAX_SENSORS), the summary of
  // the last such cast (pinned) and its completion event
  void* na_scratch = nullptr;
  Plan* na_plan = nullptr;
  Summary* na_sum = nullptr;
  hipEvent_t na_ev = nullptr;
  bool na_live = false;   // may still be running (scene or sensor changes wait for it)
  bool na_check = false;  // its summary has not been inspected by grca_synchronize
  uint32_t na_nids = 0;
  uint32_t na_ids[GRCA_NOALLOC_MAX_SENSORS] = {};
};

namespace {

grca_status fail(const grca_context* ctx, grca_status code, const std::string& msg) {
  if (ctx) const_cast<grca_context*>(ctx)->err = msg;
  return code;
}

#define HIPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail(ctx, e_ == hipErrorOutOfMemory ? GRCA_ERR_OUT_OF_MEMORY : GRCA_ERR_DEVICE, \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                       \
  } while (0)

#define GUARD(...)                                                       \
  try {                                                                  \
    __VA_ARGS__                                                          \
  } catch (const std::bad_alloc&) {                                      \
    return fail(ctx, GRCA_ERR_OUT_OF_MEMORY, "host allocation failed"); \
  } catch (...) {                                                        \
    return fail(ctx, GRCA_ERR_DEVICE, "unexpected exception");          \
  }

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Device bytes of one work-queue slot: the item and its first candidate index.
constexpr uint64_t ITEM_BYTES = sizeof(Item) + sizeof(uint32_t);

void free_items(grca_workspace* ws) {
  dfree(ws->items);
  dfree(ws->item_cs);
  ws->item_cap = 0;
}

// Grow the workspace buffers.  Only called while no cast is in flight on it.
grca_status ws_reserve(grca_context* ctx, grca_workspace* ws, uint64_t rays, uint64_t items,
                       uint64_t large, uint32_t nsens, uint32_t nscenes, uint64_t scratch,
                       uint64_t outs) {
  if (rays > ws->key_cap) {
    dfree(ws->keys);
    ws->key_cap = 0;
    HIPCHK(dmalloc(&ws->keys, rays));
    ws->key_cap = rays;
  }
  // queues are NSHARD equal regions
  items = (items + NSHARD - 1) / NSHARD * NSHARD;
  large = (large + NSHARD - 1) / NSHARD * NSHARD;
  if (items > ws->item_cap) {
    free_items(ws);
    HIPCHK(dmalloc(&ws->items, items));
    HIPCHK(dmalloc(&ws->item_cs, items));
    ws->item_cap = items;
  }
  if (large > ws->large_cap) {
    dfree(ws->large);
    ws->large_cap = 0;
    HIPCHK(dmalloc(&ws->large, large));
    ws->large_cap = large;
  }
  if (nsens > ws->sens_cap) {
    dfree(ws->dsens);
    if (ws->dsens_host) (void)hipHostFree(ws->dsens_host);
    ws->dsens_host = nullptr;
    ws->sens_cap = 0;
    HIPCHK(dmalloc(&ws->dsens, (size_t)RING * nsens));
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&ws->dsens_host),
                         (size_t)RING * nsens * sizeof(DevSensor)));
    ws->sens_cap = nsens;
  }
  if (nscenes > ws->scene_cap) {
    dfree(ws->dscenes);
    if (ws->dscenes_host) (void)hipHostFree(ws->dscenes_host);
    ws->dscenes_host = nullptr;
    ws->scene_cap = 0;
    HIPCHK(dmalloc(&ws->dscenes, (size_t)RING * nscenes));
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&ws->dscenes_host),
                         (size_t)RING * nscenes * sizeof(DevScene)));
    ws->scene_cap = nscenes;
  }
  if (scratch > ws->scratch_cap) {
    dfree(ws->scratch);
    ws->scratch_cap = 0;
    HIPCHK(dmalloc(&ws->scratch, scratch));
    ws->scratch_cap = scratch;
  }
  if (outs > ws->out_cap) {
    dfree(ws->out_dist);
    dfree(ws->out_tri);
    ws->out_cap = 0;
    HIPCHK(dmalloc(&ws->out_dist, outs));
    HIPCHK(dmalloc(&ws->out_tri, outs));
    ws->out_cap = outs;
  }
  ws->bytes = ws->key_cap * 8 + ws->item_cap * ITEM_BYTES + ws->large_cap * sizeof(Item) +
              (uint64_t)RING * (ws->sens_cap * sizeof(DevSensor) + ws->scene_cap * sizeof(DevScene)) +
              ws->scratch_cap * sizeof(Statics) + ws->out_cap * 8 + sizeof(Counters);
  return GRCA_OK;
}

grca_status ws_init(grca_context* ctx, grca_workspace* ws) {
  ws->ctx = ctx;
  HIPCHK(dmalloc(&ws->cnt, 1));
  HIPCHK(hipMemset(ws->cnt, 0, sizeof(Counters)));  // the sticky record starts clear
  HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&ws->cnt_host), RING * sizeof(Summary)));
  std::memset(ws->cnt_host, 0, RING * sizeof(Summary));
  for (int i = 0; i < RING; ++i) HIPCHK(hipEventCreateWithFlags(&ws->ev[i], hipEventDisableTiming));
  return GRCA_OK;
}

void ws_free(grca_workspace* ws) {
  if (!ws) return;
  for (int i = 0; i < RING; ++i)
    if (ws->ev[i]) (void)hipEventSynchronize(ws->ev[i]);
  dfree(ws->keys); free_items(ws); dfree(ws->large); dfree(ws->cnt);
  dfree(ws->dsens); dfree(ws->dscenes); dfree(ws->scratch);
  dfree(ws->out_dist); dfree(ws->out_tri);
  if (ws->cnt_host) (void)hipHostFree(ws->cnt_host);
  if (ws->dsens_host) (void)hipHostFree(ws->dsens_host);
  if (ws->dscenes_host) (void)hipHostFree(ws->dscenes_host);
  for (int i = 0; i < RING; ++i)
    if (ws->ev[i]) (void)hipEventDestroy(ws->ev[i]);
  delete ws;
}


// A sensor's device record, without the per-cast fields (output offset,
// scene slot, single-sided flag).
DevSensor sensor_record(const SensorData& S) {
  DevSensor d{};
  for (int c = 0; c < 3; ++c) {
    d.o[c] = S.desc.origin[c]; d.f[c] = S.desc.forward[c];
    d.r[c] = S.desc.right[c]; d.u[c] = S.desc.up[c];
  }
  d.dmin = S.desc.range_min;
  d.dmax = S.desc.range_max;
  d.gamma = S.desc.num_channels;
  d.chi = S.desc.rays_per_channel;
  d.wrap = S.wrap ? 1u : 0u;
  d.lut_size = S.lut_size;
  const double theta0 = -std::floor(d.chi / 2.0) * S.dtheta;
  d.theta_start = (float)theta0;
  d.inv_dtheta = (float)(1.0 / S.dtheta);
  d.period_idx = (float)(kTwoPi / S.dtheta);
  d.theta_start_d = theta0;
  d.inv_dtheta_d = 1.0 / S.dtheta;
  d.period_idx_d = kTwoPi / S.dtheta;
  d.chan = S.chan; d.chan_d = S.chan_d; d.sin_tab = S.sin_tab; d.bins = S.lut; d.az = S.az;
  d.mask = S.mask;
  d.elev0 = S.elev0;
  d.inv_delev = S.inv_delev;
  d.elev_tol = S.elev_tol;
  d.cull_dmax = d.dmax * (1.0f + 1e-5f) + 1e-6f;
  d.in_dmax = d.dmax * (1.0f - 1e-5f);
  d.in_dmin = d.dmin * (1.0f + 1e-5f);
  d.elev_m = 3e-5f + d.elev_tol;
  d.last_chan = (float)(d.gamma - 1u);
  d.elev0_g = d.elev0 * d.inv_delev;
  d.az_noise = S.az_noise;
  d.el_noise = S.el_noise;
  d.fov_mode = 0;
  if (!S.wrap) {
    const double m = 1e-4 + S.az_noise;
    const double lo = theta0 - m, hi = theta0 + (d.chi - 1u) * S.dtheta + m;
    if (hi - lo < kTwoPi) {
      d.fov_mode = hi - lo <= 0.5 * kTwoPi ? 1u : 2u;
      d.fov_n[0] = (float)-std::sin(lo);
      d.fov_n[1] = (float)std::cos(lo);
      d.fov_n[2] = (float)std::sin(hi);
      d.fov_n[3] = (float)-std::cos(hi);
    }
  }
  d.upright = std::fabs(d.u[0]) + std::fabs(d.u[1]) <= 1e-4f && d.u[2] > 0.0f ? 1u : 0u;
  d.pad_[0] = d.pad_[1] = d.pad_[2] = 0u;
  d.key_offset = 0;
  d.scene = 0;
  d.cull_back = 0;
  d.lossy = 0;
  d.eps_area = 0.0f;
  return d;
}

// Allocates nothing when P's vectors already hold n sensors and n scenes
// (the context's temporaries are reserved for the largest cast).
grca_status make_plan(grca_context* ctx, const uint32_t* ids, uint32_t n, uint32_t block,
                      Plan& P, uint32_t flags = 0) {
  if (n == 0) return fail(ctx, GRCA_ERR_INVALID_ARG, "num_sensors must be >= 1");
  if (n > MAX_CAST_SENSORS) return fail(ctx, GRCA_ERR_INVALID_ARG, "at most 4096 sensors per cast");
  std::vector<const SensorData*>& sd = ctx->plan_sd;
  std::vector<uint64_t>& offs = ctx->plan_off;
  sd.resize(n);
  offs.resize(n);
  uint64_t off = 0;
  for (uint32_t i = 0; i < n; ++i) {
    auto it = ctx->sensors.find(ids[i]);
    if (it == ctx->sensors.end())
      return fail(ctx, GRCA_ERR_NOT_FOUND, "unknown sensor id " + std::to_string(ids[i]));
    sd[i] = &it->second;
    if (!ctx->scenes.count(sd[i]->desc.scene_id))
      return fail(ctx, GRCA_ERR_NOT_FOUND,
                  "sensor " + std::to_string(ids[i]) + " observes unknown scene " +
                      std::to_string(sd[i]->desc.scene_id));
    offs[i] = off;
    off += (uint64_t)sd[i]->desc.num_channels * sd[i]->desc.rays_per_channel;
  }
  if (off >= (1ull << 32)) return fail(ctx, GRCA_ERR_INVALID_ARG, "more than 2^32 rays in one cast");
  P.rays = off;
  P.pairs = 0;
  std::vector<uint32_t>& order = ctx->plan_order;
  order.resize(n);
  for (uint32_t i = 0; i < n; ++i) order[i] = i;
  // grouped by scene, in call order within a scene (std::sort works in place)
  std::sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
    const uint32_t sa = sd[a]->desc.scene_id, sb = sd[b]->desc.scene_id;
    return sa != sb ? sa < sb : a < b;
  });
  P.sens.resize(n);
  P.scenes.clear();
  uint64_t tiles = 0;
  for (uint32_t k = 0; k < n; ++k) {
    const uint32_t i = order[k];
    const SensorData& S = *sd[i];
    const uint32_t sid = S.desc.scene_id;
    if (k == 0 || sd[order[k - 1]]->desc.scene_id != sid) {
      const SceneData& sc = ctx->scenes.at(sid);
      DevScene ds{};
      ds.v = sc.v; ds.soup = sc.soup; ds.n_soup = sc.n_soup; ds.idx = sc.idx; ds.orig = sc.orig;
      ds.tsph = sc.tsph; ds.gsph = sc.gsph; ds.n_pre = sc.n_pre;
      ds.ntri = sc.ntri;
      ds.tile_start = tiles;
      ds.sensor_begin = k;
      ds.sensor_end = k;
      tiles += (sc.ntri + BOUNDS_TILE - 1) / BOUNDS_TILE;
      P.scenes.push_back(ds);
    }
    DevScene& cur = P.scenes.back();
    cur.sensor_end = k + 1;
    P.pairs += cur.ntri;
    DevSensor d = sensor_record(S);
    d.key_offset = (uint32_t)offs[i];
    d.scene = (uint32_t)(P.scenes.size() - 1);
    d.cull_back = 0;
    d.lossy = flags & (GRCA_LOSSY_AREA | GRCA_LOSSY_CSPAN | GRCA_LOSSY_RSPAN);
    d.eps_area = ctx->opt.eps_area;
    if (flags & GRCA_CULL_BACKFACE) {
      const float* f = S.desc.forward;
      const float* r = S.desc.right;
      const float* u = S.desc.up;
      const double det = (double)f[0] * ((double)r[1] * u[2] - (double)r[2] * u[1]) -
                         (double)f[1] * ((double)r[0] * u[2] - (double)r[2] * u[0]) +
                         (double)f[2] * ((double)r[0] * u[1] - (double)r[1] * u[0]);
      d.cull_back = det > 0.0 ? 1 : -1;
    }
    P.sens[k] = d;
  }
  if (tiles >= (1ull << 32)) return fail(ctx, GRCA_ERR_INVALID_ARG, "too many triangles in one cast");
  P.total_tiles = (uint32_t)tiles;
  return GRCA_OK;
}

uint32_t persist_blocks(const grca_context* ctx) {
  const uint32_t waves = (uint32_t)std::max(1, ctx->num_cu) * ctx->opt.persist_waves_cu;
  return std::max(1u, waves / 4u);
}

// The device buffers one cast's kernels use.  Queues are NSHARD regions of
// icap (items and their candidate starts) and lcap (large records) entries.
struct CastBufs {
  const DevSensor* dsens;
  const DevScene* dscenes;
  unsigned long long* keys;
  Item* items;
  uint32_t* item_cs;
  uint32_t icap;
  Item* large;
  uint32_t lcap;
  Counters* cnt;
  Statics* statics;  // all-pairs only: one per triangle of the largest scene
};

// The kernel sequence of one cast: key init, then bounds + binning,
// expansion and intersection (or the all-pairs reference), then resolve.
// With `ev` (culled casts), events ev[0..4] are recorded after init, bounds,
// expansion, intersection and resolve.
grca_status launch_cast(grca_context* ctx, const Plan& P, const CastBufs& B, float* dist,
                        uint32_t* tri, uint32_t flags, hipStream_t st,
                        hipEvent_t* ev = nullptr) {
  const grca_options& o = ctx->opt;
  const uint32_t n = (uint32_t)P.rays;
  HIPCHK(launch_init(B.keys, n, B.cnt, st));
  if (ev) HIPCHK(hipEventRecord(ev[0], st));
  if (flags & GRCA_CAST_ALL_PAIRS) {
    for (uint32_t k = 0; k < P.sens.size(); ++k) {
      const DevSensor& d = P.sens[k];
      HIPCHK(launch_allpairs(B.dscenes, B.dsens, k, P.scenes[d.scene].ntri, d.gamma * d.chi,
                             B.statics, B.keys, st));
    }
  } else {
    HIPCHK(launch_bounds(B.dscenes, (uint32_t)P.scenes.size(), P.total_tiles, o.bounds_block,
                         B.dsens, o.small_channels, o.small_rays, B.items, B.item_cs, B.icap,
                         B.large, B.lcap, B.cnt, o.group_cull, o.inline_max,
                         (flags & (GRCA_LOSSY_CSPAN | GRCA_LOSSY_RSPAN)) != 0,
                         B.keys, st));
    if (ev) HIPCHK(hipEventRecord(ev[1], st));
    const uint32_t pb = persist_blocks(ctx);
    HIPCHK(launch_expand(B.dscenes, B.dsens, B.large, B.items, B.item_cs, B.icap, B.lcap,
                         o.row_chunk, B.cnt, pb, st));
    if (ev) HIPCHK(hipEventRecord(ev[2], st));
    HIPCHK(launch_isect(B.dscenes, B.dsens, (uint32_t)P.sens.size(), B.items, B.item_cs, B.icap,
                        o.isect_ticket, B.cnt, B.keys, pb, st));
    if (ev) HIPCHK(hipEventRecord(ev[3], st));
  }
  HIPCHK(launch_resolve(B.keys, n, dist, tri, B.cnt, st));
  if (ev) HIPCHK(hipEventRecord(ev[4], st));
  return GRCA_OK;
}

// The buffers of workspace `ws` for a cast whose descriptors are in ring
// slot `slot`.
CastBufs ws_bufs(grca_workspace* ws, uint32_t slot) {
  return CastBufs{ws->dsens + (size_t)slot * ws->sens_cap,
                  ws->dscenes + (size_t)slot * ws->scene_cap,
                  ws->keys, ws->items, ws->item_cs,
                  (uint32_t)(ws->item_cap / NSHARD), ws->large,
                  (uint32_t)(ws->large_cap / NSHARD), ws->cnt, ws->scratch};
}

// Enqueue the kernels of one cast into ring slot `slot` (the slot is free and
// the workspace buffers are large enough).
grca_status enqueue_kernels(grca_context* ctx, grca_workspace* ws, uint32_t slot, const Plan& P,
                            float* dist, uint32_t* tri, uint32_t flags, hipStream_t st) {
  DevSensor* dsens = ws->dsens + (size_t)slot * ws->sens_cap;
  DevScene* dscenes = ws->dscenes + (size_t)slot * ws->scene_cap;
  std::memcpy(ws->dsens_host + (size_t)slot * ws->sens_cap, P.sens.data(),
              P.sens.size() * sizeof(DevSensor));
  std::memcpy(ws->dscenes_host + (size_t)slot * ws->scene_cap, P.scenes.data(),
              P.scenes.size() * sizeof(DevScene));
  HIPCHK(hipMemcpyAsync(dsens, ws->dsens_host + (size_t)slot * ws->sens_cap,
                        P.sens.size() * sizeof(DevSensor), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(dscenes, ws->dscenes_host + (size_t)slot * ws->scene_cap,
                        P.scenes.size() * sizeof(DevScene), hipMemcpyHostToDevice, st));
  const grca_status rc = launch_cast(ctx, P, ws_bufs(ws, slot), dist, tri, flags, st);
  if (rc != GRCA_OK) return rc;
  HIPCHK(hipMemcpyAsync(ws->cnt_host + slot, &ws->cnt->sum, sizeof(Summary),
                        hipMemcpyDeviceToHost, st));
  HIPCHK(hipEventRecord(ws->ev[slot], st));
  return GRCA_OK;
}

// New queue capacities after an overflow, from the requested counts.
// A shard that overflowed asked for max_*_shard slots; every shard gets that
// many plus a quarter.  A large-queue overflow also grows the item queue (the
// dropped large records' rows were never counted).
grca_status grown_caps(grca_context* ctx, const Summary& c, uint64_t& items, uint64_t& large) {
  const uint64_t want_i = NSHARD * ((uint64_t)c.max_items_shard + c.max_items_shard / 4 + 1024);
  const uint64_t want_l = NSHARD * ((uint64_t)c.max_large_shard + c.max_large_shard / 4 + 16);
  if (c.overflow & 2u) {
    large = std::max<uint64_t>(large * 2, want_l);
    items = std::max<uint64_t>(items * 2, want_i);
  }
  if (c.overflow & 1u) items = std::max<uint64_t>(items * 2, want_i);
  if (c.overflow & 4u)
    return fail(ctx, GRCA_ERR_CAPACITY, "candidate pairs of one queue shard exceed 2^32");
  if (items > 0xFFFFFFF0ull || large > 0xFFFFFFF0ull)
    return fail(ctx, GRCA_ERR_CAPACITY, "work queue would exceed 2^32 entries");
  return GRCA_OK;
}

grca_status ws_quiesce(grca_context* ctx, grca_workspace* ws) {
  for (int i = 0; i < RING; ++i)
    if (ws->rec[i].live) HIPCHK(hipEventSynchronize(ws->ev[i]));
  return GRCA_OK;
}

// Wait for every cast in flight on `ws`; recast (synchronously, with grown
// queues) every one whose queues overflowed.
grca_status ws_drain(grca_context* ctx, grca_workspace* ws) {
  grca_status rc = ws_quiesce(ctx, ws);
  if (rc != GRCA_OK) return rc;
  for (uint32_t k = 0; k < (uint32_t)RING; ++k) {
    const uint32_t slot = (ws->next_slot + k) % RING;  // oldest first
    CastRecord& R = ws->rec[slot];
    if (!R.live) continue;
    int attempt = 0;
    if (ws->cnt_host[slot].overflow) R.overflowed = 1;
    while (ws->cnt_host[slot].overflow) {
      if (++attempt > 6) {
        R.live = false;
        return fail(ctx, GRCA_ERR_CAPACITY, "work queue kept overflowing after regrowth");
      }
      uint64_t items = ws->item_cap, large = ws->large_cap;
      rc = grown_caps(ctx, ws->cnt_host[slot], items, large);
      if (rc != GRCA_OK) { R.live = false; return rc; }
      free_items(ws);
      dfree(ws->large); ws->large_cap = 0;
      rc = ws_reserve(ctx, ws, 0, items, large, 0, 0, 0, 0);
      if (rc != GRCA_OK) { R.live = false; return rc; }
      Plan P;
      rc = make_plan(ctx, R.ids.data(), (uint32_t)R.ids.size(), ctx->opt.bounds_block, P,
                     R.flags);
      if (rc != GRCA_OK) { R.live = false; return rc; }
      rc = enqueue_kernels(ctx, ws, slot, P, R.dist, R.tri, R.flags, R.st);
      if (rc != GRCA_OK) { R.live = false; return rc; }
      R.recasts++;
      HIPCHK(hipEventSynchronize(ws->ev[slot]));
    }
    R.live = false;
  }
  return GRCA_OK;
}

grca_status check_vec(const float* v, const char* name, const grca_context* ctx) {
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(v[k])) return fail(ctx, GRCA_ERR_INVALID_ARG, std::string(name) + " not finite");
  return GRCA_OK;
}

// Before a scene or sensor changes: finish every cast and frame launch still
// in flight that reads it (recasting overflowed ones with the state they were
// issued against), and, with `stale`, mark the frames that read it for
// re-capture (their graphs hold its device pointers).  scene_id / sensor_id
// of -1 match nothing.  Defined with the frames below.
grca_status settle_users(grca_context* ctx, int64_t scene_id, int64_t sensor_id, bool stale);

}  // namespace

// =============================================================== context
namespace {
// Device address of each device's no-allocation scratch array, looked up
// once per device (with that device current) by the first context on it.
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

// Set-up of the no-allocation cast (the device is current): the scratch
// array's device address, the planner's reserved temporaries, the pinned
// summary and the completion event.
grca_status noalloc_init(grca_context* ctx) {
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    void* p = ctx->device < 64 ? g_scratch_ptr[ctx->device] : nullptr;
    if (!p) {
      HIPCHK(noalloc_scratch_address(&p));
      if (!p) return fail(ctx, GRCA_ERR_DEVICE, "no device address for the scratch array");
      if (ctx->device < 64) g_scratch_ptr[ctx->device] = p;
    }
    ctx->na_scratch = p;
  }
  ctx->plan_sd.reserve(MAX_CAST_SENSORS);
  ctx->plan_off.reserve(MAX_CAST_SENSORS);
  ctx->plan_order.reserve(MAX_CAST_SENSORS);
  ctx->na_plan = new Plan();
  ctx->na_plan->sens.reserve(GRCA_NOALLOC_MAX_SENSORS);
  ctx->na_plan->scenes.reserve(GRCA_NOALLOC_MAX_SENSORS);
  HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&ctx->na_sum), sizeof(Summary)));
  std::memset(ctx->na_sum, 0, sizeof(Summary));
  HIPCHK(hipEventCreateWithFlags(&ctx->na_ev, hipEventDisableTiming));
  return GRCA_OK;
}
}  // namespace

extern "C" grca_status grca_create(int hip_device, grca_context** out) {
  grca_context* ctx = nullptr;
  if (!out) return GRCA_ERR_INVALID_ARG;
  *out = nullptr;
  try {
    ctx = new grca_context();
  } catch (...) {
    return GRCA_ERR_OUT_OF_MEMORY;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) {
    delete ctx;
    return GRCA_ERR_DEVICE;
  }
  if (hipSetDevice(hip_device) != hipSuccess) { delete ctx; return GRCA_ERR_DEVICE; }
  ctx->device = hip_device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) { delete ctx; return GRCA_ERR_DEVICE; }
  ctx->num_cu = prop.multiProcessorCount;
  ctx->opt.small_channels = 8;
  ctx->opt.small_rays = 64;
  ctx->opt.row_chunk = 256;
  ctx->opt.bounds_block = 256;
  ctx->opt.persist_waves_cu = 16;
  ctx->opt.group_cull = 1;
  ctx->opt.inline_max = 0;
  ctx->opt.isect_ticket = 4096;
  ctx->opt.eps_area = 1e-6f;
  ctx->opt.item_capacity = 1u << 20;
  ctx->opt.large_capacity = 1u << 16;
  ctx->def_ws = new grca_workspace();
  if (ws_init(ctx, ctx->def_ws) != GRCA_OK || noalloc_init(ctx) != GRCA_OK) {
    grca_destroy(ctx);
    return GRCA_ERR_DEVICE;
  }
  ctx->workspaces.insert(ctx->def_ws);
  *out = ctx;
  return GRCA_OK;
}

extern "C" void grca_destroy(grca_context* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  ws_free(ctx->def_ws);
  for (auto& kv : ctx->scenes) free_scene(kv.second);
  for (auto& kv : ctx->sensors) free_sensor(kv.second);
  if (ctx->na_sum) (void)hipHostFree(ctx->na_sum);
  if (ctx->na_ev) (void)hipEventDestroy(ctx->na_ev);
  delete ctx->na_plan;
  delete ctx;
}

extern "C" const char* grca_last_error(const grca_context* ctx) {
  return ctx ? ctx->err.c_str() : "null context";
}

// =============================================================== scenes
grca_status reorder_scene(grca_context* ctx, SceneData& sc, hipStream_t st) {
  const hipError_t e = reorder_scene_dev(sc, st);
  if (e != hipSuccess)
    return fail(ctx, GRCA_ERR_DEVICE, std::string("triangle tile order: ") + hipGetErrorString(e));
  return GRCA_OK;
}

extern "C" grca_status grca_scene_update(grca_context* ctx, uint32_t scene_id,
                                         const float* vertices_xyz, uint32_t num_vertices,
                                         const uint32_t* indices, uint32_t num_triangles,
                                         uint32_t flags, void* hip_stream) {
  if (!ctx) return GRCA_ERR_INVALID_ARG;
  GUARD({
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t st = as_stream(hip_stream);
    const bool dev = flags & GRCA_MEM_DEVICE;
    const bool vonly = flags & GRCA_UPDATE_VERTICES_ONLY;
    if (num_vertices > 0 && !vertices_xyz) return fail(ctx, GRCA_ERR_INVALID_ARG, "vertices is NULL");
    // the kernels address indices (12 B per triangle) and vertices (16 B
    // each) by 32-bit byte offsets
    if (num_triangles >= (1u << 28)) return fail(ctx, GRCA_ERR_INVALID_ARG, "too many triangles");
    if (num_vertices >= (1u << 28)) return fail(ctx, GRCA_ERR_INVALID_ARG, "too many vertices");
    auto it = ctx->scenes.find(scene_id);
    if (vonly) {
      if (it == ctx->scenes.end()) return fail(ctx, GRCA_ERR_NOT_FOUND, "unknown scene");
      if (it->second.nv != num_vertices)
        return fail(ctx, GRCA_ERR_INVALID_ARG, "vertex count differs from the scene's");
    } else if (num_triangles > 0 && !indices) {
      return fail(ctx, GRCA_ERR_INVALID_ARG, "indices is NULL");
    }
    // validate before touching the stored scene
    if (!dev) {
      for (uint64_t i = 0; i < 3ull * num_vertices; ++i)
        if (!std::isfinite(vertices_xyz[i]))
          return fail(ctx, GRCA_ERR_INVALID_ARG, "non-finite vertex coordinate");
      if (!vonly)
        for (uint64_t i = 0; i < 3ull * num_triangles; ++i)
          if (indices[i] >= num_vertices)
            return fail(ctx, GRCA_ERR_INVALID_ARG, "index out of range");
    } else {
      uint32_t* bad = nullptr;
      HIPCHK(dmalloc(&bad, 1));
      uint32_t zero = 0, hbad = 0;
      HIPCHK(hipMemcpyAsync(bad, &zero, 4, hipMemcpyHostToDevice, st));
      HIPCHK(launch_validate(vertices_xyz, num_vertices, vonly ? nullptr : indices,
                             vonly ? 0 : 3ull * num_triangles, bad, st));
      HIPCHK(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      dfree(bad);
      if (hbad & 1u) return fail(ctx, GRCA_ERR_INVALID_ARG, "non-finite vertex coordinate");
      if (hbad & 2u) return fail(ctx, GRCA_ERR_INVALID_ARG, "index out of range");
    }
    if (it != ctx->scenes.end()) {
      // a topology update reallocates the scene; a vertex-only update keeps its buffers
      grca_status rs = settle_users(ctx, scene_id, -1, !vonly);
      if (rs != GRCA_OK) return rs;
    }
    SceneData fresh;
    SceneData& sc = (it == ctx->scenes.end()) ? fresh : it->second;
    const bool realloc_v = sc.nv != num_vertices || !sc.v;
    if (!vonly && it != ctx->scenes.end()) {
      // topology change drops dynamic-geometry declarations
      HIPCHK(hipStreamSynchronize(st));
      SceneData keep;
      keep.v = sc.v; keep.idx = sc.idx; keep.orig = sc.orig;
      keep.nv = sc.nv; keep.ntri = sc.ntri;
      sc.v = nullptr; sc.idx = nullptr; sc.orig = nullptr;
      free_scene(sc);
      sc = SceneData();
      sc.v = keep.v; sc.idx = keep.idx; sc.orig = keep.orig;
      sc.nv = keep.nv; sc.ntri = keep.ntri;
    }
    if (realloc_v) {
      HIPCHK(hipStreamSynchronize(st));
      dfree(sc.v);
      HIPCHK(dmalloc(&sc.v, std::max(1u, num_vertices)));
    }
    float* tmp = nullptr;
    if (num_vertices) {
      const float* src = vertices_xyz;
      if (!dev) {
        HIPCHK(dmalloc(&tmp, 3ull * num_vertices));
        HIPCHK(hipMemcpyAsync(tmp, vertices_xyz, 12ull * num_vertices, hipMemcpyHostToDevice, st));
        src = tmp;
      }
      HIPCHK(launch_pad(src, num_vertices, sc.v, st));
    }
    if (!vonly) {
      if (sc.ntri != num_triangles || !sc.idx) {
        HIPCHK(hipStreamSynchronize(st));
        dfree(sc.idx);
        dfree(sc.orig);
        HIPCHK(dmalloc(&sc.idx, 3ull * std::max(1u, num_triangles)));
        HIPCHK(dmalloc(&sc.orig, std::max(1u, num_triangles)));
      }
      if (num_triangles)
        HIPCHK(hipMemcpyAsync(sc.idx, indices, 12ull * num_triangles,
                              dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
      HIPCHK(launch_iota(sc.orig, num_triangles, st));
      sc.ntri = num_triangles;
    }
    sc.nv = num_vertices;
    if (!vonly) {
      grca_status rc = reorder_scene(ctx, sc, st);
      if (rc != GRCA_OK) return rc;
    } else {
      HIPCHK(refresh_soup(sc, st));
    }
    if (tmp) {
      HIPCHK(hipStreamSynchronize(st));
      dfree(tmp);
    }
    if (it == ctx->scenes.end()) ctx->scenes.emplace(scene_id, fresh);
    return GRCA_OK;
  })
}

extern "C" grca_status grca_scene_download(grca_context* ctx, uint32_t scene_id,
                                           float* vertices_xyz_host, void* hip_stream) {
  if (!ctx) return GRCA_ERR_INVALID_ARG;
  GUARD({
    auto it = ctx->scenes.find(scene_id);
    if (it == ctx->scenes.end()) return fail(ctx, GRCA_ERR_NOT_FOUND, "unknown scene");
    if (!vertices_xyz_host) return fail(ctx, GRCA_ERR_INVALID_ARG, "NULL output");
    HIPCHK(hipSetDevice(ctx->device));
    const SceneData& sc = it->second;
    const size_t nv = sc.nv;
    std::vector<float4> v(nv);
    hipStream_t st = as_stream(hip_stream);
    if (nv) HIPCHK(hipMemcpyAsync(v.data(), sc.v, 16 * nv, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (size_t i = 0; i < nv; ++i) {
      vertices_xyz_host[3 * i] = v[i].x;
      vertices_xyz_host[3 * i + 1] = v[i].y;
      vertices_xyz_host[3 * i + 2] = v[i].z;
    }
    return GRCA_OK;
  })
}

extern "C" grca_status grca_scene_release(grca_context* ctx, uint32_t scene_id) {
  if (!ctx) return GRCA_ERR_INVALID_ARG;
  GUARD({
    auto it = ctx->scenes.find(scene_id);
    if (it == ctx->scenes.end()) return fail(ctx, GRCA_ERR_NOT_FOUND, "unknown scene");
    HIPCHK(hipSetDevice(ctx->device));
    grca_status rs = settle_users(ctx, scene_id, -1, true);
    if (rs != GRCA_OK) return rs;
    HIPCHK(hipDeviceSynchronize());
    free_scene(it->second);
    ctx->scenes.erase(it);
    return GRCA_OK;
  })
}

namespace {
grca_status check_ranges(grca_context* ctx, const SceneData& sc, uint32_t n, const uint32_t* st,
                         const uint32_t* ct) {
  std::vector<std::pair<uint64_t, uint64_t>> r(n);
  for (uint32_t i = 0; i < n; ++i) {
    if ((uint64_t)st[i] + ct[i] > sc.nv)
      return fail(ctx, GRCA_ERR_INVALID_ARG, "vertex range outside the scene");
    r[i] = {st[i], (uint64_t)st[i] + ct[i]};
  }
  std::sort(r.begin(), r.end());
  for (uint32_t i = 1; i < n; ++i)
    if (r[i].first < r[i - 1].second) return fail(ctx, GRCA_ERR_INVALID_ARG, "vertex ranges overlap");
  return GRCA_OK;
}

grca_status ensure_pose_block(grca_context* ctx, SceneData& sc) {
  const size_t bytes = 8 + 48ull * sc.n_inst;
  if (bytes == sc.pose_bytes && sc.pose_in) return GRCA_OK;
  dfree(sc.pose_in);
  if (sc.pose_stage) (void)hipHostFree(sc.pose_stage);
  sc.pose_stage = nullptr;
  HIPCHK(dmalloc(&sc.pose_in, (bytes + 7) / 8));
  HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&sc.pose_stage), bytes));
  std::memset(sc.pose_stage, 0, bytes);
  if (!sc.pose_ev) HIPCHK(hipEventCreateWithFlags(&sc.pose_ev, hipEventDisableTiming));
  sc.pose_bytes = bytes;
  return GRCA_OK;
}

std::vector<PoseBlock> pose_blocks(uint32_t kind, const std::vector<uint32_t>& starts,
                                   const std::vector<uint32_t>& counts) {
  std::vector<PoseBlock> out;
  uint32_t rest = 0;
  for (size_t g = 0; g < starts.size(); ++g) {
    for (uint32_t o = 0; o < counts[g]; o += POSE_BLOCK_VERTS) {
      PoseBlock b{};
      b.kind = kind;
      b.group = (uint32_t)g;
      b.v_begin = starts[g] + o;
      b.count = std::min(POSE_BLOCK_VERTS, counts[g] - o);
      b.rest_begin = rest + o;
      out.push_back(b);
    }
    rest += counts[g];
  }
  return out;
}
}  // namespace

extern "C" grca_status grca_scene_set_rigid(grca_context* ctx, uint32_t scene_id,
                                            uint32_t num_instances, const uint32_t* vertex_start,
                                            const uint32_t* vertex_count, void* hip_stream) {
  if (!ctx) return GRCA_ERR_INVALID_ARG;
  GUARD({
    HIPCHK(hipSetDevice(ctx->device));
    auto it = ctx->scenes.find(scene_id);
    if (it == ctx->scenes.end()) return fail(ctx, GRCA_ERR_NOT_FOUND, "unknown scene");
    if (num_instances && (!vertex_start || !vertex_count))
      return fail(ctx, GRCA_ERR_INVALID_ARG, "NULL instance arrays");
    SceneData& sc = it->second;
    grca_status rc = check_ranges(ctx, sc, num_instances, vertex_start, vertex_count);
    if (rc != GRCA_OK) return rc;
    rc = settle_users(ctx, scene_id, -1, true);
    if (rc != GRCA_OK) return rc;
    hipStream_t st = as_stream(hip_stream);
    HIPCHK(hipStreamSynchronize(st));
    dfree(sc.rr_x); dfree(sc.rr_y); dfree(sc.rr_z); dfree(sc.rigid_blocks);
    sc.inst_start.assign(vertex_start, vertex_start + num_instances);
    sc.inst_count.assign(vertex_count, vertex_count + num_instances);
    sc.n_inst = num_instances;
    uint64_t total = 0;
    for (uint32_t i = 0; i < num_instances; ++i) total += vertex_count[i];
    HIPCHK(dmalloc(&sc.rr_x, std::max<uint64_t>(total, 1)));
    HIPCHK(dmalloc(&sc.rr_y, std::max<uint64_t>(total, 1)));
    HIPCHK(dmalloc(&sc.rr_z, std::max<uint64_t>(total, 1)));
    uint64_t r = 0;
    for (uint32_t i = 0; i < num_instances; ++i) {
      HIPCHK(launch_split(sc.v + vertex_start[i], vertex_count[i], sc.rr_x + r, sc.rr_y + r,
                          sc.rr_z + r, st));
      r += vertex_count[i];
    }
    std::vector<PoseBlock> pb = pose_blocks(0, sc.inst_start, sc.inst_count);
    sc.n_rigid_blocks = (uint32_t)pb.size();
    HIPCHK(dmalloc(&sc.rigid_blocks, std::max<size_t>(pb.size(), 1)));
    if (!pb.empty())
      HIPCHK(hipMemcpy(sc.rigid_blocks, pb.data(), pb.size() * sizeof(PoseBlock), hipMemcpyHostToDevice));
    rc = ensure_pose_block(ctx, sc);
    if (rc != GRCA_OK) return rc;
    HIPCHK(hipStreamSynchronize(st));
    return reorder_scene(ctx, sc, st);
  })
}

extern "C" grca_status grca_scene_set_deform(grca_context* ctx, uint32_t scene_id,
                                             uint32_t num_groups, const grca_deform_group* groups,
                                             const float* normals_xyz, const float* phases,
                                             void* hip_stream) {
  if (!ctx) return GRCA_ERR_INVALID_ARG;
  GUARD({
    HIPCHK(hipSetDevice(ctx->device));
    auto it = ctx->scenes.find(scene_id);
    if (it == ctx->scenes.end()) return fail(ctx, GRCA_ERR_NOT_FOUND, "unknown scene");
    if (num_groups && (!groups || !normals_xyz || !phases))
      return fail(ctx, GRCA_ERR_INVALID_ARG, "NULL deform arrays");
    SceneData& sc = it->second;
    std::vector<uint32_t> st_v(num_groups), ct_v(num_groups);
    uint64_t total = 0;
    for (uint32_t g = 0; g < num_groups; ++g) {
      st_v[g] = groups[g].vertex_start;
      ct_v[g] = groups[g].vertex_count;
      if (!std::isfinite(groups[g].amplitude) || !std::isfinite(groups[g].omega))
        return fail(ctx, GRCA_ERR_INVALID_ARG, "non-finite deform parameter");
      total += ct_v[g];
    }
    grca_status rc = check_ranges(ctx, sc, num_groups, st_v.data(), ct_v.data());
    if (rc != GRCA_OK) return rc;
    for (uint64_t i = 0; i < 3 * total; ++i)
      if (!std::isfinite(normals_xyz[i])) return fail(ctx, GRCA_ERR_INVALID_ARG, "non-finite normal");
    for (uint64_t i = 0; i < total; ++i)
      if (!std::isfinite(phases[i])) return fail(ctx, GRCA_ERR_INVALID_ARG, "non-finite phase");
    rc = settle_users(ctx, scene_id, -1, true);
    if (rc != GRCA_OK) return rc;
    hipStream_t st = as_stream(hip_stream);
    HIPCHK(hipStreamSynchronize(st));
    dfree(sc.dr_x); dfree(sc.dr_y); dfree(sc.dr_z);
    dfree(sc.dn_x); dfree(sc.dn_y); dfree(sc.dn_z); dfree(sc.dphase);
    dfree(sc.deform_blocks); dfree(sc.dparams);
    sc.groups.assign(groups, groups + num_groups);
    sc.n_groups = num_groups;
    const uint64_t nt = std::max<uint64_t>(total, 1);
    HIPCHK(dmalloc(&sc.dr_x, nt)); HIPCHK(dmalloc(&sc.dr_y, nt)); HIPCHK(dmalloc(&sc.dr_z, nt));
    HIPCHK(dmalloc(&sc.dn_x, nt)); HIPCHK(dmalloc(&sc.dn_y, nt)); HIPCHK(dmalloc(&sc.dn_z, nt));
    HIPCHK(dmalloc(&sc.dphase, nt));
    std::vector<float> nx(total), ny(total), nz(total);
    for (uint64_t i = 0; i < total; ++i) {
      nx[i] = normals_xyz[3 * i]; ny[i] = normals_xyz[3 * i + 1]; nz[i] = normals_xyz[3 * i + 2];
    }
    if (total) {
      HIPCHK(hipMemcpy(sc.dn_x, nx.data(), 4 * total, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(sc.dn_y, ny.data(), 4 * total, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(sc.dn_z, nz.data(), 4 * total, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(sc.dphase, phases, 4 * total, hipMemcpyHostToDevice));
    }
    uint64_t r = 0;
    for (uint32_t g = 0; g < num_groups; ++g) {
      HIPCHK(launch_split(sc.v + st_v[g], ct_v[g], sc.dr_x + r, sc.dr_y + r, sc.dr_z + r, st));
      r += ct_v[g];
    }
    std::vector<PoseBlock> pb = pose_blocks(1, st_v, ct_v);
    sc.n_deform_blocks = (uint32_t)pb.size();
    HIPCHK(dmalloc(&sc.deform_blocks, std::max<size_t>(pb.size(), 1)));
    if (!pb.empty())
      HIPCHK(hipMemcpy(sc.deform_blocks, pb.data(), pb.size() * sizeof(PoseBlock), hipMemcpyHostToDevice));
    std::vector<DeformParam> dp(num_groups);
    for (uint32_t g = 0; g < num_groups; ++g) dp[g] = DeformParam{groups[g].amplitude, groups[g].omega};
    HIPCHK(dmalloc(&sc.dparams, std::max<size_t>(dp.size(), 1)));
    if (!dp.empty())
      HIPCHK(hipMemcpy(sc.dparams, dp.data(), dp.size() * sizeof(DeformParam), hipMemcpyHostToDevice));
    rc = ensure_pose_block(ctx, sc);
    if (rc != GRCA_OK) return rc;
    HIPCHK(hipStreamSynchronize(st));
    return reorder_scene(ctx, sc, st);
  })
}

namespace {
grca_status enqueue_pose_kernels(grca_context* ctx, SceneData& sc, hipStream_t st) {
  HIPCHK(launch_pose(sc.rigid_blocks, sc.n_rigid_blocks, sc.rr_x, sc.rr_y, sc.rr_z,
                     sc.deform_blocks, sc.n_deform_blocks, sc.dr_x, sc.dr_y, sc.dr_z, sc.dn_x,
                     sc.dn_y, sc.dn_z, sc.dphase, sc.dparams, sc.pose_in, sc.v, st));
  return GRCA_OK;
}

grca_status stage_pose(grca_context* ctx, SceneData& sc, const float* mats, double time,
                       bool dev_mats, hipStream_t st) {
  if (!sc.pose_in) return GRCA_OK;
  if (sc.n_inst && !mats) return fail(ctx, GRCA_ERR_INVALID_ARG, "instance matrices required");
  HIPCHK(hipEventSynchronize(sc.pose_ev));
  std::memcpy(sc.pose_stage, &time, 8);
  if (sc.n_inst && !dev_mats) {
    for (uint64_t i = 0; i < 12ull * sc.n_inst; ++i)
      if (!std::isfinite(mats[i])) return fail(ctx, GRCA_ERR_INVALID_ARG, "non-finite matrix");
    std::memcpy(sc.pose_stage + 8, mats, 48ull * sc.n_inst);
    HIPCHK(hipMemcpyAsync(sc.pose_in, sc.pose_stage, sc.pose_bytes, hipMemcpyHostToDevice, st));
  } else {
    HIPCHK(hipMemcpyAsync(sc.pose_in, sc.pose_stage, 8, hipMemcpyHostToDevice, st));
    if (sc.n_inst)
      HIPCHK(hipMemcpyAsync(reinterpret_cast<unsigned char*>(sc.pose_in) + 8, mats,
                            48ull * sc.n_inst, hipMemcpyDeviceToDevice, st));
  }
  HIPCHK(hipEventRecord(sc.pose_ev, st));
  return GRCA_OK;
}
}  // namespace

extern "C" grca_status grca_scene_pose(grca_context* ctx, uint32_t scene_id,
                                       const float* instance_matrices, double time_s,
                                       uint32_t flags, void* hip_stream) {
  if (!ctx) return GRCA_ERR_INVALID_ARG;
  GUARD({
    HIPCHK(hipSetDevice(ctx->device));
    auto it = ctx->scenes.find(scene_id);
    if (it == ctx->scenes.end()) return fail(ctx, GRCA_ERR_NOT_FOUND, "unknown scene");
    if (!std::isfinite(time_s)) return fail(ctx, GRCA_ERR_INVALID_ARG, "time not finite");
    SceneData& sc = it->second;
    hipStream_t st = as_stream(hip_stream);
    grca_status rc = settle_users(ctx, scene_id, -1, false);
    if (rc != GRCA_OK) return rc;
    rc = stage_pose(ctx, sc, instance_matrices, time_s, flags & GRCA_MEM_DEVICE, st);
    if (rc != GRCA_OK) return rc;
    return enqueue_pose_kernels(ctx, sc, st);
  })
}

// =============================================================== sensors
extern "C" grca_status grca_sensor_config(grca_context* ctx, uint32_t sensor_id,
                                          const grca_sensor_desc* s) {
  if (!ctx) return GRCA_ERR_INVALID_ARG;
  GUARD({
    if (!s) return fail(ctx, GRCA_ERR_INVALID_ARG, "NULL descriptor");
    grca_status rc;
    if ((rc = check_vec(s->origin, "origin", ctx)) != GRCA_OK) return rc;
    if ((rc = check_vec(s->forward, "forward", ctx)) != GRCA_OK) return rc;
    if ((rc = check_vec(s->right, "right", ctx)) != GRCA_OK) return rc;
    if ((rc = check_vec(s->up, "up", ctx)) != GRCA_OK) return rc;
    const float* B[3] = {s->forward, s->right, s->up};
    for (int a = 0; a < 3; ++a)
      for (int b = a; b < 3; ++b) {
        const double d = (double)B[a][0] * B[b][0] + (double)B[a][1] * B[b][1] +
                         (double)B[a][2] * B[b][2];
        if (std::fabs(d - (a == b ? 1.0 : 0.0)) > 1e-6)
          return fail(ctx, GRCA_ERR_INVALID_ARG, "basis not orthonormal within 1e-6");
      }
    if (s->num_channels < 1 || s->num_channels > 65535)
      return fail(ctx, GRCA_ERR_INVALID_ARG, "num_channels outside [1, 65535]");
    if (s->rays_per_channel < 1 || s->rays_per_channel > 65535)
      return fail(ctx, GRCA_ERR_INVALID_ARG, "rays_per_channel outside [1, 65535]");
    if (!s->channel_elevation_rad) return fail(ctx, GRCA_ERR_INVALID_ARG, "NULL elevation table");
    const double half_pi = 1.5707963267948966;
    for (uint32_t j = 0; j < s->num_channels; ++j) {
      const float e = s->channel_elevation_rad[j];
      if (!std::isfinite(e) || std::fabs((double)e) > half_pi + 1e-6)
        return fail(ctx, GRCA_ERR_INVALID_ARG, "elevation outside [-pi/2, pi/2]");
      if (j && !(e > s->channel_elevation_rad[j - 1]))
        return fail(ctx, GRCA_ERR_INVALID_ARG, "elevations not strictly ascending");
    }
    if (!(s->fov_rad > 0.0f) || (double)s->fov_rad > kTwoPi + 1e-6)
      return fail(ctx, GRCA_ERR_INVALID_ARG, "fov outside (0, 2 pi]");
    if (!(s->range_min > 0.0f) || !(s->range_max >= s->range_min) || !std::isfinite(s->range_max))
      return fail(ctx, GRCA_ERR_INVALID_ARG, "need 0 < range_min <= range_max < inf");
    float az_noise = 0.0f;
    if (s->azimuth_offset_rad) {
      const double step = (double)s->fov_rad / (double)s->rays_per_channel;
      for (uint32_t r = 0; r < s->rays_per_channel; ++r) {
        const float a = s->azimuth_offset_rad[r];
        if (!std::isfinite(a) || std::fabs((double)a) > step)
          return fail(ctx, GRCA_ERR_INVALID_ARG, "azimuth offset not finite or beyond one ray step");
        az_noise = std::max(az_noise, std::fabs(a));
      }
      az_noise = az_noise * 1.0001f + 1e-7f;
    }
    float el_noise = 0.0f;
    if (s->channel_elevation_offset_rad) {
      for (uint32_t j = 0; j < s->num_channels; ++j) {
        const float o = s->channel_elevation_offset_rad[j];
        if (!std::isfinite(o) ||
            std::fabs((double)s->channel_elevation_rad[j] + (double)o) > half_pi + 1e-6)
          return fail(ctx, GRCA_ERR_INVALID_ARG,
                      "elevation offset not finite or the perturbed elevation beyond pi/2");
        el_noise = std::max(el_noise, std::fabs(o));
      }
      el_noise = el_noise * 1.0001f + 1e-7f;
    }
    HIPCHK(hipSetDevice(ctx->device));
    SensorData sd;
    sd.desc = *s;
    sd.elev.assign(s->channel_elevation_rad, s->channel_elevation_rad + s->num_channels);
    {
      // the channel elevations as a uniform grid (exact for evenly spaced
      // tables) and the largest distance of a channel from it
      const uint32_t g = s->num_channels;
      const double e0 = (double)sd.elev[0];
      const double step = g > 1 ? ((double)sd.elev[g - 1] - e0) / (double)(g - 1) : 1.0;
      double tol = 0.0;
      for (uint32_t j = 0; j < g; ++j)
        tol = std::max(tol, std::fabs((double)sd.elev[j] - (e0 + (double)j * step)));
      sd.elev0 = sd.elev[0];
      sd.inv_delev = (float)(1.0 / step);
      // + the FP32 rounding of 1 / step over the whole table, + the largest
      // elevation offset (the perturbed channels lie within it of the grid)
      sd.elev_tol = (float)(tol * (1.0 + 1e-6) + 1e-6) + el_noise;
    }
    sd.desc.channel_elevation_rad = nullptr;
    sd.dtheta = (double)s->fov_rad / (double)s->rays_per_channel;
    sd.wrap = std::fabs((double)s->fov_rad - kTwoPi) <= 1e-6;
    sd.az_noise = az_noise;
    sd.el_noise = el_noise;
    sd.desc.channel_elevation_offset_rad = nullptr;
    sd.desc.azimuth_offset_rad = nullptr;
    sd.desc.ray_mask = nullptr;
    // bins of at most a quarter of the smallest gap between channel sines, so
    // that a channel search is almost always one table load (at most 16384)
    double min_gap = 2.0;
    for (uint32_t j = 0; j + 1 < s->num_channels; ++j)
      min_gap = std::min(min_gap, std::sin((double)s->channel_elevation_rad[j + 1]) -
                                      std::sin((double)s->channel_elevation_rad[j]));
    double want = std::max(512.0, 4.0 * s->num_channels);
    if (min_gap > 0.0) want = std::max(want, std::ceil(8.0 / min_gap));
    sd.lut_size = (uint32_t)std::min(want, 16384.0);
    const uint32_t g = s->num_channels, c = s->rays_per_channel;
    auto cleanup = [&]() { free_sensor(sd); };
    hipError_t e = hipSuccess;
    float* elev_d = nullptr;
    float* off_d = nullptr;
    float* eoff_d = nullptr;
    if ((e = dmalloc(&sd.chan, g)) != hipSuccess || (e = dmalloc(&sd.chan_d, g)) != hipSuccess ||
        (e = dmalloc(&sd.sin_tab, g)) != hipSuccess || (e = dmalloc(&sd.az, c)) != hipSuccess ||
        (e = dmalloc(&sd.lut, sd.lut_size)) != hipSuccess || (e = dmalloc(&elev_d, g)) != hipSuccess ||
        (s->azimuth_offset_rad && (e = dmalloc(&off_d, c)) != hipSuccess) ||
        (s->channel_elevation_offset_rad && (e = dmalloc(&eoff_d, g)) != hipSuccess) ||
        (s->ray_mask && (e = dmalloc(&sd.mask, (size_t)g * c)) != hipSuccess)) {
      cleanup();
      dfree(elev_d);
      dfree(off_d);
      dfree(eoff_d);
      return fail(ctx, GRCA_ERR_OUT_OF_MEMORY, std::string("sensor tables: ") + hipGetErrorString(e));
    }
    e = hipMemcpy(elev_d, sd.elev.data(), 4ull * g, hipMemcpyHostToDevice);
    if (e == hipSuccess && off_d)
      e = hipMemcpy(off_d, s->azimuth_offset_rad, 4ull * c, hipMemcpyHostToDevice);
    if (e == hipSuccess && eoff_d)
      e = hipMemcpy(eoff_d, s->channel_elevation_offset_rad, 4ull * g, hipMemcpyHostToDevice);
    if (e == hipSuccess && sd.mask)
      e = hipMemcpy(sd.mask, s->ray_mask, (size_t)g * c, hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = launch_sensor_tables(elev_d, eoff_d, g, c, sd.dtheta, off_d, sd.chan, sd.chan_d, sd.sin_tab,
                               sd.az, sd.lut_size, sd.lut, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    dfree(elev_d);
    dfree(off_d);
    dfree(eoff_d);
    if (e != hipSuccess) {
      cleanup();
      return fail(ctx, GRCA_ERR_DEVICE, std::string("sensor tables: ") + hipGetErrorString(e));
    }
    auto it = ctx->sensors.find(sensor_id);
    if (it != ctx->sensors.end()) {
      const grca_status rs = settle_users(ctx, -1, sensor_id, true);
      if (rs != GRCA_OK) {
        cleanup();
        return rs;
      }
      HIPCHK(hipDeviceSynchronize());
      free_sensor(it->second);
      it->second = sd;
    } else {
      ctx->sensors.emplace(sensor_id, sd);
    }
    return GRCA_OK;
  })
}

extern "C" grca_status grca_sensor_release(grca_context* ctx, uint32_t sensor_id) {
  if (!ctx) return GRCA_ERR_INVALID_ARG;
  GUARD({
    auto it = ctx->sensors.find(sensor_id);
    if (it == ctx->sensors.end()) return fail(ctx, GRCA_ERR_NOT_FOUND, "unknown sensor");
    HIPCHK(hipSetDevice(ctx->device));
    grca_status rs = settle_users(ctx, -1, sensor_id, true);
    if (rs != GRCA_OK) return rs;
    HIPCHK(hipDeviceSynchronize());
    free_sensor(it->second);
    ctx->sensors.erase(it);
    return GRCA_OK;
  })
}

// =============================================================== casting
namespace {
grca_status cast_on(grca_context* ctx, grca_workspace* ws, const uint32_t* ids, uint32_t n,
                    float* out_dist, uint32_t* out_tri, uint32_t flags, hipStream_t st) {
  if (n && !ids) return fail(ctx, GRCA_ERR_INVALID_ARG, "NULL sensor id list");
  Plan P;
  grca_status rc = make_plan(ctx, ids, n, ctx->opt.bounds_block, P, flags);
  if (rc != GRCA_OK) return rc;
  if (ws->fixed && P.rays > ws->key_cap)
    return fail(ctx, GRCA_ERR_CAPACITY, "cast has more rays than the workspace holds");
  const bool dev = flags & GRCA_MEM_DEVICE;
  uint64_t scratch = 0;
  if (flags & GRCA_CAST_ALL_PAIRS)
    for (const DevScene& s : P.scenes) scratch = std::max<uint64_t>(scratch, s.ntri);
  const uint64_t want_items = ws->item_cap ? ws->item_cap : ctx->opt.item_capacity;
  const uint64_t want_large = ws->large_cap ? ws->large_cap : ctx->opt.large_capacity;
  const bool grow = P.rays > ws->key_cap || want_items > ws->item_cap ||
                    want_large > ws->large_cap || P.sens.size() > ws->sens_cap ||
                    P.scenes.size() > ws->scene_cap || scratch > ws->scratch_cap ||
                    (!dev && P.rays > ws->out_cap);
  const uint32_t slot = ws->next_slot;
  if (grow || ws->rec[slot].live) {
    // buffers are about to change, or the ring wrapped: finish everything in flight
    rc = ws_drain(ctx, ws);
    if (rc != GRCA_OK) return rc;
    rc = ws_reserve(ctx, ws, std::max<uint64_t>(P.rays, 1), want_items, want_large,
                    (uint32_t)P.sens.size(), (uint32_t)P.scenes.size(), scratch,
                    dev ? 0 : P.rays);
    if (rc != GRCA_OK) return rc;
  } else if (ws->last_slot >= 0 && ws->rec[ws->last_slot].live && ws->last_stream != st) {
    // another stream used these buffers last: order after it on the device
    HIPCHK(hipStreamWaitEvent(st, ws->ev[ws->last_slot], 0));
  }
  float* dist = dev ? out_dist : (out_dist ? ws->out_dist : nullptr);
  uint32_t* tri = dev ? out_tri : (out_tri ? ws->out_tri : nullptr);
  CastRecord& R = ws->rec[slot];
  R.ids.assign(ids, ids + n);
  R.dist = dist;
  R.tri = tri;
  R.flags = flags;
  R.st = st;
  R.rays = P.rays;
  R.pairs = P.pairs;
  R.recasts = 0;
  R.overflowed = 0;
  rc = enqueue_kernels(ctx, ws, slot, P, dist, tri, flags, st);
  if (rc != GRCA_OK) return rc;
  R.live = true;
  ws->last_slot = (int)slot;
  ws->last_stream = st;
  ws->next_slot = (slot + 1) % RING;
  ctx->last_ws = ws;
  if (!dev) {
    rc = ws_drain(ctx, ws);
    if (rc != GRCA_OK) return rc;
    if (out_dist) HIPCHK(hipMemcpyAsync(out_dist, ws->out_dist, 4 * P.rays, hipMemcpyDeviceToHost, st));
    if (out_tri) HIPCHK(hipMemcpyAsync(out_tri, ws->out_tri, 4 * P.rays, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  return GRCA_OK;
}
}  // namespace

extern "C" grca_status grca_cast(grca_context* ctx, const uint32_t* sensor_ids,
                                 uint32_t num_sensors, float* out_distance, uint32_t* out_tri,
                                 uint32_t flags, void* hip_stream) {
  if (!ctx) return GRCA_ERR_INVALID_ARG;
  GUARD({
    HIPCHK(hipSetDevice(ctx->device));
    return cast_on(ctx, ctx->def_ws, sensor_ids, num_sensors, out_distance, out_tri, flags,
                   as_stream(hip_stream));
  })
}

extern "C" grca_status grca_synchronize(grca_context* ctx, void* hip_stream) {
  if (!ctx) return GRCA_ERR_INVALID_ARG;
  GUARD({
    HIPCHK(hipSetDevice(ctx->device));
    grca_status rc = ws_drain(ctx, ctx->def_ws);
    if (rc != GRCA_OK) return rc;
    HIPCHK(hipStreamSynchronize(as_stream(hip_stream)));
    if (ctx->na_check) {
      // the last no-allocation cast: its queues could not grow
      HIPCHK(hipEventSynchronize(ctx->na_ev));
      ctx->na_live = false;
      ctx->na_check = false;
      if (ctx->na_sum->overflow)
        return fail(ctx, GRCA_ERR_CAPACITY,
                    "a no-allocation cast overflowed its fixed work queues (its outputs are "
                    "incomplete); cast it with grca_cast, or with fewer rays");
    }
    return GRCA_OK;
  })
}

extern "C" grca_status grca_cast_noalloc(grca_context* ctx, const uint32_t* sensor_ids,
                                         uint32_t num_sensors, float* out_distance_dev,
                                         uint32_t* out_tri_dev, uint32_t flags,
                                         void* hip_stream) {
  if (!ctx) return GRCA_ERR_INVALID_ARG;
  GUARD({
    HIPCHK(hipSetDevice(ctx->device));
    if (!ctx->na_scratch) return fail(ctx, GRCA_ERR_DEVICE, "no-allocation scratch not set up");
    if (!(flags & GRCA_MEM_DEVICE))
      return fail(ctx, GRCA_ERR_INVALID_ARG, "grca_cast_noalloc writes device outputs only");
    if (flags & ~(GRCA_MEM_DEVICE | GRCA_CULL_BACKFACE))
      return fail(ctx, GRCA_ERR_INVALID_ARG,
                  "grca_cast_noalloc accepts GRCA_MEM_DEVICE and GRCA_CULL_BACKFACE only");
    if (num_sensors > GRCA_NOALLOC_MAX_SENSORS)
      return fail(ctx, GRCA_ERR_INVALID_ARG, "grca_cast_noalloc takes at most 64 sensors");
    if (num_sensors && !sensor_ids) return fail(ctx, GRCA_ERR_INVALID_ARG, "NULL sensor id list");
    Plan& P = *ctx->na_plan;
    grca_status rc = make_plan(ctx, sensor_ids, num_sensors, ctx->opt.bounds_block, P, flags);
    if (rc != GRCA_OK) return rc;
    // carve the scratch array: counters, descriptors, keys, then the queues
    const size_t total = GRCA_NOALLOC_SCRATCH_BYTES;
    unsigned char* const base = static_cast<unsigned char*>(ctx->na_scratch);
    size_t used = 0;
    auto take = [&](size_t bytes) {
      unsigned char* p = base + used;
      used += (bytes + 255u) & ~(size_t)255u;
      return p;
    };
    Counters* cnt = reinterpret_cast<Counters*>(take(sizeof(Counters)));
    DevSensor* dsens = reinterpret_cast<DevSensor*>(take(sizeof(DevSensor) * GRCA_NOALLOC_MAX_SENSORS));
    DevScene* dscenes = reinterpret_cast<DevScene*>(take(sizeof(DevScene) * GRCA_NOALLOC_MAX_SENSORS));
    const size_t key_bytes = ((size_t)P.rays * 8u + 255u) & ~(size_t)255u;
    if (used + key_bytes + GRCA_NOALLOC_MIN_QUEUE_BYTES > total)
      return fail(ctx, GRCA_ERR_CAPACITY,
                  "grca_cast_noalloc: " + std::to_string(P.rays) +
                      " rays leave too little of the 64 MiB scratch array for the work queues");
    unsigned long long* keys = reinterpret_cast<unsigned long long*>(take(key_bytes));
    // an eighth of the rest for large records, the remainder for items and
    // their candidate starts; both within the options' capacities
    uint64_t lcap = std::min<uint64_t>(ctx->opt.large_capacity, (total - used) / 8u / sizeof(Item));
    lcap = std::max<uint64_t>(lcap / NSHARD, 1u) * NSHARD;
    Item* large = reinterpret_cast<Item*>(take(lcap * sizeof(Item)));
    uint64_t icap = std::min<uint64_t>(ctx->opt.item_capacity, (total - used - 768u) / ITEM_BYTES);
    icap = std::max<uint64_t>(icap / NSHARD, 1u) * NSHARD;
    Item* items = reinterpret_cast<Item*>(take(icap * sizeof(Item)));
    uint32_t* item_cs = reinterpret_cast<uint32_t*>(take(icap * sizeof(uint32_t)));
    if (used > total) return fail(ctx, GRCA_ERR_CAPACITY, "grca_cast_noalloc: scratch layout");
    hipStream_t st = as_stream(hip_stream);
    // the cast's descriptors travel in kernel arguments (no host staging)
    HIPCHK(launch_put(dsens, P.sens.data(), P.sens.size() * sizeof(DevSensor), st));
    HIPCHK(launch_put(dscenes, P.scenes.data(), P.scenes.size() * sizeof(DevScene), st));
    const CastBufs B{dsens, dscenes, keys, items, item_cs, (uint32_t)(icap / NSHARD),
                     large, (uint32_t)(lcap / NSHARD), cnt, nullptr};
    rc = launch_cast(ctx, P, B, out_distance_dev, out_tri_dev, flags, st);
    if (rc != GRCA_OK) return rc;
    HIPCHK(hipMemcpyAsync(ctx->na_sum, &cnt->sum, sizeof(Summary), hipMemcpyDeviceToHost, st));
    HIPCHK(hipEventRecord(ctx->na_ev, st));
    ctx->na_live = true;
    ctx->na_check = true;
    ctx->na_nids = num_sensors;
    std::copy(sensor_ids, sensor_ids + num_sensors, ctx->na_ids);
    return GRCA_OK;
  })
}

namespace {
grca_status stats_of(grca_context* ctx, grca_workspace* ws, grca_stats* out) {
  std::memset(out, 0, sizeof(*out));
  if (!ws || ws->last_slot < 0) return GRCA_OK;
  HIPCHK(hipSetDevice(ctx->device));
  const int slot = ws->last_slot;
  const bool was_live = ws->rec[slot].live;
  grca_status rc = ws_drain(ctx, ws);
  if (rc != GRCA_OK) return rc;
  if (!was_live) HIPCHK(hipEventSynchronize(ws->ev[slot]));
  const Summary& c = ws->cnt_host[slot];
  const CastRecord& R = ws->rec[slot];
  out->rays = R.rays;
  out->pairs_tested = R.pairs;
  out->rect_items = c.n_items >= c.n_rows ? c.n_items - c.n_rows : 0;
  out->large_records = c.n_large;
  out->row_items = c.n_rows;
  out->rtic = c.rtic;
  out->recasts = R.recasts;
  out->overflowed = R.overflowed;
  out->pairs_evaluated = c.pairs;
  out->sphere_tests = c.tests;
  out->atomics = c.atomics;
  return GRCA_OK;
}
}  // namespace

extern "C" grca_status grca_last_stats(grca_context* ctx, grca_stats* out) {
  if (!ctx || !out) return GRCA_ERR_INVALID_ARG;
  GUARD({ return stats_of(ctx, ctx->last_ws, out); })
}

extern "C" grca_status grca_workspace_stats(grca_context* ctx, grca_workspace* ws,
                                            grca_stats* out) {
  if (!ctx || !ws || ws->ctx != ctx || !out) return GRCA_ERR_INVALID_ARG;
  GUARD({ return stats_of(ctx, ws, out); })
}

// =============================================================== options
extern "C" grca_status grca_get_options(const grca_context* ctx, grca_options* out) {
  if (!ctx || !out) return GRCA_ERR_INVALID_ARG;
  *out = ctx->opt;
  return GRCA_OK;
}

extern "C" grca_status grca_set_options(grca_context* ctx, const grca_options* o) {
  if (!ctx || !o) return GRCA_ERR_INVALID_ARG;
  if (o->small_channels < 1 || o->small_channels > 255)
    return fail(ctx, GRCA_ERR_INVALID_ARG, "small_channels outside [1, 255]");
  if (o->small_rays < 1 || o->small_rays > 65535)
    return fail(ctx, GRCA_ERR_INVALID_ARG, "small_rays outside [1, 65535]");
  if (o->row_chunk < 1 || o->row_chunk > 65535)
    return fail(ctx, GRCA_ERR_INVALID_ARG, "row_chunk outside [1, 65535]");
  const uint32_t b = o->bounds_block;
  if (b != 64 && b != 128 && b != 256 && b != 512 && b != 1024)
    return fail(ctx, GRCA_ERR_INVALID_ARG, "bounds_block must be 64, 128, 256, 512 or 1024");
  if (o->group_cull > 1) return fail(ctx, GRCA_ERR_INVALID_ARG, "group_cull must be 0 or 1");
  if (o->inline_max > 4096) return fail(ctx, GRCA_ERR_INVALID_ARG, "inline_max outside [0, 4096]");
  if (o->isect_ticket < 64 || o->isect_ticket > (1u << 20) || o->isect_ticket % 64 != 0)
    return fail(ctx, GRCA_ERR_INVALID_ARG, "isect_ticket must be a multiple of 64 in [64, 2^20]");
  if (!std::isfinite(o->eps_area) || o->eps_area < 0.0f)
    return fail(ctx, GRCA_ERR_INVALID_ARG, "eps_area must be finite and >= 0");
  if (o->persist_waves_cu < 1 || o->persist_waves_cu > 32)
    return fail(ctx, GRCA_ERR_INVALID_ARG, "persist_waves_cu outside [1, 32]");
  if (o->item_capacity < 64 || o->item_capacity > 0xFFFFFFF0ull ||
      o->large_capacity < 64 || o->large_capacity > 0xFFFFFFF0ull)
    return fail(ctx, GRCA_ERR_INVALID_ARG, "queue capacities outside [64, 2^32)");
  ctx->opt = *o;
  return GRCA_OK;
}

// =============================================================== workspaces
extern "C" grca_status grca_workspace_create(grca_context* ctx, uint64_t max_rays,
                                             uint64_t item_capacity, grca_workspace** out,
                                             uint64_t* bytes_out) {
  if (!ctx || !out) return GRCA_ERR_INVALID_ARG;
  GUARD({
    *out = nullptr;
    if (max_rays == 0 || max_rays >= (1ull << 32))
      return fail(ctx, GRCA_ERR_INVALID_ARG, "max_rays outside [1, 2^32)");
    if (item_capacity < 64 || item_capacity > 0xFFFFFFF0ull)
      return fail(ctx, GRCA_ERR_INVALID_ARG, "item_capacity outside [64, 2^32)");
    HIPCHK(hipSetDevice(ctx->device));
    grca_workspace* ws = new grca_workspace();
    grca_status rc = ws_init(ctx, ws);
    if (rc == GRCA_OK)
      rc = ws_reserve(ctx, ws, max_rays, item_capacity,
                      std::max<uint64_t>(item_capacity / 16, 4096), 64, 16, 0, 0);
    if (rc != GRCA_OK) {
      ws_free(ws);
      return rc;
    }
    ws->fixed = true;
    ctx->workspaces.insert(ws);
    *out = ws;
    if (bytes_out) *bytes_out = ws->bytes;
    return GRCA_OK;
  })
}

extern "C" void grca_workspace_destroy(grca_workspace* ws) {
  if (!ws) return;
  if (ws->ctx) {
    if (ws->ctx->last_ws == ws) ws->ctx->last_ws = nullptr;
    ws->ctx->workspaces.erase(ws);
    (void)hipSetDevice(ws->ctx->device);
  }
  ws_free(ws);
}

extern "C" grca_status grca_cast_ws(grca_context* ctx, grca_workspace* ws,
                                    const uint32_t* sensor_ids, uint32_t num_sensors,
                                    float* out_distance_dev, uint32_t* out_tri_dev,
                                    void* hip_stream) {
  if (!ctx || !ws || ws->ctx != ctx) return GRCA_ERR_INVALID_ARG;
  GUARD({
    HIPCHK(hipSetDevice(ctx->device));
    return cast_on(ctx, ws, sensor_ids, num_sensors, out_distance_dev, out_tri_dev,
                   GRCA_MEM_DEVICE, as_stream(hip_stream));
  })
}

extern "C" grca_status grca_workspace_synchronize(grca_context* ctx, grca_workspace* ws,
                                                  void* hip_stream) {
  if (!ctx || !ws || ws->ctx != ctx) return GRCA_ERR_INVALID_ARG;
  GUARD({
    HIPCHK(hipSetDevice(ctx->device));
    (void)hip_stream;
    return ws_drain(ctx, ws);
  })
}

// =============================================================== frames
namespace {
// The frame's stage sequence on stream `st`; with `ev` non-null an event is
// recorded before the first stage and after each stage.
grca_status enqueue_frame(grca_context* ctx, grca_frame* fr, const Plan& P, hipStream_t st,
                          hipEvent_t* ev) {
  SceneData& sc = ctx->scenes.at(fr->scene_id);
  grca_workspace* ws = fr->ws;
  if (ev) HIPCHK(hipEventRecord(ev[0], st));
  if (sc.pose_in) {
    grca_status rc = enqueue_pose_kernels(ctx, sc, st);
    if (rc != GRCA_OK) return rc;
  }
  if (ev) HIPCHK(hipEventRecord(ev[1], st));
  // the frame's tables live in ring slot 0
  const grca_status rc = launch_cast(ctx, P, ws_bufs(ws, 0), fr->out_dist, fr->out_tri,
                                     GRCA_MEM_DEVICE, st, ev ? ev + 2 : nullptr);
  if (rc != GRCA_OK) return rc;
  HIPCHK(hipMemcpyAsync(ws->cnt_host, &ws->cnt->sum, sizeof(Summary), hipMemcpyDeviceToHost, st));
  return GRCA_OK;
}

grca_status capture_one(grca_context* ctx, grca_frame* fr, const Plan& P) {
  hipStream_t st = fr->cap_stream;
  HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  const grca_status erc = enqueue_frame(ctx, fr, P, st, nullptr);
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(st, &g);
  if (erc != GRCA_OK) {
    if (g) (void)hipGraphDestroy(g);
    return erc;
  }
  if (e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(ctx, GRCA_ERR_DEVICE, std::string("frame capture: ") + hipGetErrorString(e2));
  }
  fr->graph = g;
  HIPCHK(hipGraphInstantiate(&fr->exec, g, nullptr, nullptr, 0));
  return GRCA_OK;
}

void destroy_graphs(grca_frame* fr) {
  if (fr->exec) (void)hipGraphExecDestroy(fr->exec);
  if (fr->graph) (void)hipGraphDestroy(fr->graph);
  fr->exec = nullptr;
  fr->graph = nullptr;
}

grca_status frame_plan(grca_context* ctx, grca_frame* fr, Plan& P) {
  for (uint32_t id : fr->ids) {
    auto it = ctx->sensors.find(id);
    if (it != ctx->sensors.end() && it->second.desc.scene_id != fr->scene_id)
      return fail(ctx, GRCA_ERR_INVALID_ARG,
                  "frame sensor " + std::to_string(id) + " no longer observes the frame's scene");
  }
  return make_plan(ctx, fr->ids.data(), (uint32_t)fr->ids.size(), ctx->opt.bounds_block, P);
}

grca_status capture_frame(grca_context* ctx, grca_frame* fr) {
  destroy_graphs(fr);
  Plan P;
  grca_status rc = frame_plan(ctx, fr, P);
  if (rc != GRCA_OK) return rc;
  grca_workspace* ws = fr->ws;
  rc = ws_quiesce(ctx, ws);
  if (rc != GRCA_OK) return rc;
  // size every buffer before capture (no allocation inside the graph)
  rc = ws_reserve(ctx, ws, P.rays, ws->item_cap ? ws->item_cap : ctx->opt.item_capacity,
                  ws->large_cap ? ws->large_cap : ctx->opt.large_capacity,
                  (uint32_t)P.sens.size(), (uint32_t)P.scenes.size(), 0, 0);
  if (rc != GRCA_OK) return rc;
  // the frame's tables live in ring slot 0 and never change
  std::memcpy(ws->dsens_host, P.sens.data(), P.sens.size() * sizeof(DevSensor));
  std::memcpy(ws->dscenes_host, P.scenes.data(), P.scenes.size() * sizeof(DevScene));
  HIPCHK(hipMemcpy(ws->dsens, ws->dsens_host, P.sens.size() * sizeof(DevSensor), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(ws->dscenes, ws->dscenes_host, P.scenes.size() * sizeof(DevScene), hipMemcpyHostToDevice));
  rc = capture_one(ctx, fr, P);
  if (rc != GRCA_OK) return rc;
  CastRecord& R = ws->rec[0];
  R.ids = fr->ids;
  R.rays = P.rays;
  R.pairs = P.pairs;
  R.dist = fr->out_dist;
  R.tri = fr->out_tri;
  R.flags = GRCA_MEM_DEVICE;
  return GRCA_OK;
}
// Wait for the frame's launches in flight and look at the sticky overflow
// record they left.  Launches that overflowed dropped work: the queues are
// grown and the graph re-captured; if the last launch overflowed it is run
// again (its pose inputs are still in place), and earlier ones, whose outputs
// have been overwritten, are counted in `lost` for grca_frame_synchronize.
grca_status frame_settle(grca_context* ctx, grca_frame* fr, hipStream_t st) {
  grca_workspace* ws = fr->ws;
  CastRecord& R = ws->rec[0];
  if (!R.live) return GRCA_OK;
  for (int attempt = 0; attempt < 7; ++attempt) {
    HIPCHK(hipEventSynchronize(ws->ev[0]));
    const Summary c = ws->cnt_host[0];
    if (!c.sticky.overflow) {
      R.live = false;
      return GRCA_OK;
    }
    fr->lost += c.sticky.casts - (c.overflow ? 1u : 0u);
    R.overflowed += c.sticky.casts;
    Summary want = c;
    want.overflow = c.sticky.overflow;
    want.max_items_shard = c.sticky.max_items_shard;
    want.max_large_shard = c.sticky.max_large_shard;
    uint64_t items = ws->item_cap, large = ws->large_cap;
    grca_status rc = grown_caps(ctx, want, items, large);
    if (rc != GRCA_OK) { R.live = false; return rc; }
    free_items(ws);
    dfree(ws->large); ws->large_cap = 0;
    rc = ws_reserve(ctx, ws, 0, items, large, 0, 0, 0, 0);
    if (rc != GRCA_OK) { R.live = false; return rc; }
    rc = capture_frame(ctx, fr);
    if (rc != GRCA_OK) { R.live = false; return rc; }
    fr->stale = false;
    HIPCHK(launch_fill(reinterpret_cast<uint32_t*>(&ws->cnt->sticky),
                       (uint32_t)(sizeof(Sticky) / sizeof(uint32_t)), 0u, st));
    if (!c.overflow) {  // the last launch was complete
      HIPCHK(hipStreamSynchronize(st));
      R.live = false;
      return GRCA_OK;
    }
    R.recasts++;
    HIPCHK(hipGraphLaunch(fr->exec, st));
    HIPCHK(hipEventRecord(ws->ev[0], st));
    R.st = st;
  }
  R.live = false;
  return fail(ctx, GRCA_ERR_CAPACITY, "frame queue kept overflowing after regrowth");
}

// A frame whose inputs were reallocated is re-captured before it runs again.
grca_status frame_refresh(grca_context* ctx, grca_frame* fr) {
  if (!fr->stale) return GRCA_OK;
  const grca_status rc = capture_frame(ctx, fr);
  if (rc == GRCA_OK) fr->stale = false;
  return rc;
}

grca_status settle_users(grca_context* ctx, int64_t scene_id, int64_t sensor_id, bool stale) {
  auto reads = [&](const std::vector<uint32_t>& ids) {
    for (uint32_t id : ids) {
      if ((int64_t)id == sensor_id) return true;
      if (scene_id < 0) continue;
      auto it = ctx->sensors.find(id);
      if (it != ctx->sensors.end() && (int64_t)it->second.desc.scene_id == scene_id) return true;
    }
    return false;
  };
  for (grca_workspace* ws : ctx->workspaces) {
    bool busy = false;
    for (int i = 0; i < RING && !busy; ++i) busy = ws->rec[i].live && reads(ws->rec[i].ids);
    if (!busy) continue;
    const grca_status rc = ws_drain(ctx, ws);
    if (rc != GRCA_OK) return rc;
  }
  if (ctx->na_live) {
    const std::vector<uint32_t> na(ctx->na_ids, ctx->na_ids + ctx->na_nids);
    if (reads(na)) {
      HIPCHK(hipEventSynchronize(ctx->na_ev));
      ctx->na_live = false;
    }
  }
  for (grca_frame* fr : ctx->frames) {
    if ((int64_t)fr->scene_id != scene_id && !reads(fr->ids)) continue;
    const grca_status rc = frame_settle(ctx, fr, fr->ws->rec[0].st);
    if (rc != GRCA_OK) return rc;
    if (stale) fr->stale = true;
  }
  return GRCA_OK;
}
}  // namespace

extern "C" grca_status grca_frame_create(grca_context* ctx, uint32_t scene_id,
                                         const uint32_t* sensor_ids, uint32_t num_sensors,
                                         float* out_distance_dev, uint32_t* out_tri_dev,
                                         grca_frame** out) {
  if (!ctx || !out) return GRCA_ERR_INVALID_ARG;
  GUARD({
    *out = nullptr;
    HIPCHK(hipSetDevice(ctx->device));
    if (!ctx->scenes.count(scene_id)) return fail(ctx, GRCA_ERR_NOT_FOUND, "unknown scene");
    if (num_sensors == 0 || !sensor_ids) return fail(ctx, GRCA_ERR_INVALID_ARG, "no sensors");
    for (uint32_t i = 0; i < num_sensors; ++i) {
      auto it = ctx->sensors.find(sensor_ids[i]);
      if (it == ctx->sensors.end()) return fail(ctx, GRCA_ERR_NOT_FOUND, "unknown sensor");
      if (it->second.desc.scene_id != scene_id)
        return fail(ctx, GRCA_ERR_INVALID_ARG, "frame sensors must observe the frame's scene");
    }
    grca_frame* fr = new grca_frame();
    fr->ctx = ctx;
    fr->scene_id = scene_id;
    fr->ids.assign(sensor_ids, sensor_ids + num_sensors);
    fr->out_dist = out_distance_dev;
    fr->out_tri = out_tri_dev;
    fr->ws = new grca_workspace();
    grca_status rc = ws_init(ctx, fr->ws);
    if (rc == GRCA_OK && hipStreamCreateWithFlags(&fr->cap_stream, hipStreamNonBlocking) != hipSuccess)
      rc = fail(ctx, GRCA_ERR_DEVICE, "stream creation failed");
    for (int k = 0; k < 7 && rc == GRCA_OK; ++k)
      if (hipEventCreate(&fr->tev[k]) != hipSuccess)
        rc = fail(ctx, GRCA_ERR_DEVICE, "event creation failed");
    if (rc == GRCA_OK) rc = capture_frame(ctx, fr);
    if (rc != GRCA_OK) {
      grca_frame_destroy(fr);
      return rc;
    }
    ctx->frames.insert(fr);
    *out = fr;
    return GRCA_OK;
  })
}

extern "C" grca_status grca_frame_launch(grca_frame* fr, const float* instance_matrices,
                                         double time_s, void* hip_stream) {
  if (!fr || !fr->ctx) return GRCA_ERR_INVALID_ARG;
  grca_context* ctx = fr->ctx;
  GUARD({
    HIPCHK(hipSetDevice(ctx->device));
    auto it = ctx->scenes.find(fr->scene_id);
    if (it == ctx->scenes.end()) return fail(ctx, GRCA_ERR_NOT_FOUND, "frame scene was released");
    if (!std::isfinite(time_s)) return fail(ctx, GRCA_ERR_INVALID_ARG, "time not finite");
    hipStream_t st = as_stream(hip_stream);
    grca_workspace* ws = fr->ws;
    grca_status rc = frame_refresh(ctx, fr);
    if (rc != GRCA_OK) return rc;
    if (ws->rec[0].live && ws->rec[0].st != st) HIPCHK(hipStreamWaitEvent(st, ws->ev[0], 0));
    rc = stage_pose(ctx, it->second, instance_matrices, time_s, false, st);
    if (rc != GRCA_OK) return rc;
    HIPCHK(hipGraphLaunch(fr->exec, st));
    HIPCHK(hipEventRecord(ws->ev[0], st));
    ws->rec[0].live = true;
    ws->rec[0].st = st;
    ws->last_slot = 0;
    ctx->last_ws = ws;
    return GRCA_OK;
  })
}

extern "C" grca_status grca_frame_synchronize(grca_frame* fr, void* hip_stream) {
  if (!fr || !fr->ctx) return GRCA_ERR_INVALID_ARG;
  grca_context* ctx = fr->ctx;
  GUARD({
    HIPCHK(hipSetDevice(ctx->device));
    const grca_status rc = frame_settle(ctx, fr, as_stream(hip_stream));
    if (rc != GRCA_OK) return rc;
    if (fr->lost) {
      const uint32_t n = fr->lost;
      fr->lost = 0;
      return fail(ctx, GRCA_ERR_CAPACITY,
                  std::to_string(n) + " earlier launch(es) of this frame overflowed their work "
                  "queues and produced incomplete outputs; the queues have been grown");
    }
    return GRCA_OK;
  })
}

extern "C" void grca_frame_destroy(grca_frame* fr) {
  if (!fr) return;
  if (fr->ctx) {
    (void)hipSetDevice(fr->ctx->device);
    fr->ctx->frames.erase(fr);
  }
  if (fr->ws) (void)ws_quiesce(fr->ctx, fr->ws);
  destroy_graphs(fr);
  for (int k = 0; k < 7; ++k)
    if (fr->tev[k]) (void)hipEventDestroy(fr->tev[k]);
  if (fr->cap_stream) (void)hipStreamDestroy(fr->cap_stream);
  if (fr->ctx && fr->ctx->last_ws == fr->ws) fr->ctx->last_ws = nullptr;
  ws_free(fr->ws);
  delete fr;
}

extern "C" grca_status grca_frame_profile(grca_frame* fr, const float* instance_matrices,
                                          double time_s, void* hip_stream, float* ms6) {
  if (!fr || !fr->ctx || !ms6) return GRCA_ERR_INVALID_ARG;
  grca_context* ctx = fr->ctx;
  GUARD({
    HIPCHK(hipSetDevice(ctx->device));
    auto it = ctx->scenes.find(fr->scene_id);
    if (it == ctx->scenes.end()) return fail(ctx, GRCA_ERR_NOT_FOUND, "frame scene was released");
    if (!std::isfinite(time_s)) return fail(ctx, GRCA_ERR_INVALID_ARG, "time not finite");
    hipStream_t st = as_stream(hip_stream);
    grca_workspace* ws = fr->ws;
    grca_status rc = frame_refresh(ctx, fr);
    if (rc != GRCA_OK) return rc;
    if (ws->rec[0].live && ws->rec[0].st != st) HIPCHK(hipStreamWaitEvent(st, ws->ev[0], 0));
    rc = stage_pose(ctx, it->second, instance_matrices, time_s, false, st);
    if (rc != GRCA_OK) return rc;
    Plan P;
    rc = frame_plan(ctx, fr, P);
    if (rc != GRCA_OK) return rc;
    rc = enqueue_frame(ctx, fr, P, st, fr->tev);
    if (rc != GRCA_OK) return rc;
    HIPCHK(hipEventRecord(ws->ev[0], st));
    ws->rec[0].live = true;
    ws->rec[0].st = st;
    ws->last_slot = 0;
    ctx->last_ws = ws;
    HIPCHK(hipEventSynchronize(fr->tev[6]));
    for (int k = 0; k < 6; ++k) HIPCHK(hipEventElapsedTime(&ms6[k], fr->tev[k], fr->tev[k + 1]));
    return GRCA_OK;
  })
}

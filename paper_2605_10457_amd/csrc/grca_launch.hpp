// grca_launch.hpp -- host-callable launchers of the caster's kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "grca.h"
#include "grca_device.hpp"

namespace grca {

// Vertices per block of the pose kernel (256 threads, four vertices each,
// whose loads are in flight together).
constexpr uint32_t POSE_BLOCK_VERTS = 1024;

// One block of the pose kernel: up to POSE_BLOCK_VERTS vertices of one rigid
// instance (kind 0, `group` = instance index) or one deform group (kind 1).
struct PoseBlock {
  uint32_t kind;
  uint32_t group;
  uint32_t v_begin;    // first scene vertex of this block
  uint32_t count;      // vertices in this block (<= POSE_BLOCK_VERTS)
  uint32_t rest_begin; // first entry in the rest / normal / phase arrays
  uint32_t pad[3];
};

struct DeformParam {
  float amplitude;
  float omega;
};

hipError_t launch_init(unsigned long long* keys, uint32_t n, Counters* cnt, hipStream_t st);
// Queues (items, statics, large records) are NSHARD regions of `*_scap`
// entries each; `total_tiles` counts bounds tiles (BOUNDS_TILE triangles) over the cast's scenes.
// `item_cs` holds each item's first candidate index within its shard.
hipError_t launch_bounds(const DevScene* scenes, uint32_t nscenes, uint32_t total_tiles,
                         uint32_t block, const DevSensor* sens, uint32_t small_c, uint32_t small_r,
                         Item* items, uint32_t* item_cs, uint32_t item_scap, Item* large,
                         uint32_t large_scap, Counters* cnt, uint32_t group_cull,
                         uint32_t inline_max, bool lossy, unsigned long long* keys,
                         hipStream_t st);
hipError_t launch_expand(const DevScene* scenes, const DevSensor* sens, const Item* large,
                         Item* items, uint32_t* item_cs, uint32_t item_scap, uint32_t large_scap,
                         uint32_t row_chunk, Counters* cnt, uint32_t nblocks, hipStream_t st);
// intersection; its tickets are ranges of `ticket_cands` candidate pairs
hipError_t launch_isect(const DevScene* scenes, const DevSensor* sens, uint32_t nsens,
                        const Item* items, const uint32_t* item_cs, uint32_t item_scap,
                        uint32_t ticket_cands, Counters* cnt, unsigned long long* keys,
                        uint32_t nblocks, hipStream_t st);
hipError_t launch_allpairs(const DevScene* scenes, const DevSensor* sens, uint32_t sensor,
                           uint32_t ntri, uint32_t nrays, Statics* scratch,
                           unsigned long long* keys, hipStream_t st);
// also writes the cast's Summary from the queue counters
hipError_t launch_resolve(const unsigned long long* keys, uint32_t n, float* dist, uint32_t* tri,
                          Counters* cnt, hipStream_t st);
// both pose kinds in one launch: n_rigid rigid-instance blocks, then
// n_deform deform-group blocks
hipError_t launch_pose(const PoseBlock* rblocks, uint32_t n_rigid, const float* rrx,
                       const float* rry, const float* rrz, const PoseBlock* dblocks,
                       uint32_t n_deform, const float* drx, const float* dry, const float* drz,
                       const float* nx, const float* ny, const float* nz, const float* phase,
                       const DeformParam* groups, const double* pose_in, float4* v,
                       hipStream_t st);
// Per-sensor tables: chan / chan_d from the elevations plus the optional
// per-channel offsets (vertical noise), sin_tab and the lookup from the
// nominal (ascending) elevations, az from the azimuth grid plus offsets.
hipError_t launch_sensor_tables(const float* elev, const float* el_off, uint32_t gamma,
                                uint32_t chi, double dtheta, const float* az_off, float2* chan,
                                double2* chan_d, float* sin_tab, float2* az, uint32_t lut_size,
                                ChanBin* lut, hipStream_t st);
hipError_t launch_validate(const float* xyz, uint32_t nv, const uint32_t* idx, uint64_t nidx,
                           uint32_t* bad, hipStream_t st);
// the bounding spheres of the first n_pre tiles from their triangles' vertex
// records (soup): 128 per tile into tsph, one per tile into gsph
hipError_t launch_spheres(const float4* soup, uint32_t n_pre, float4* tsph, float4* gsph,
                          hipStream_t st);
// caller's packed xyz -> padded (x, y, z, 0) vertices
hipError_t launch_pad(const float* xyz, uint32_t nv, float4* v, hipStream_t st);
// padded vertices -> three coordinate arrays (rest positions of the pose step)
hipError_t launch_split(const float4* v, uint32_t n, float* x, float* y, float* z,
                        hipStream_t st);

// Tile order of a scene (grca_order.hip): rewrites idx (3 x ntri) in Morton
// order of triangle centroids within each dynamic group (vgroup[v] = group of
// vertex v) and permutes orig (caller triangle id of each slot) alike.
// Synchronises `st`; allocates and frees its own temporaries.
hipError_t order_triangles(uint32_t* idx, uint32_t* orig, uint32_t ntri, const float4* v,
                           uint32_t nv, const uint32_t* vgroup, hipStream_t st);
hipError_t launch_iota(uint32_t* a, uint32_t n, hipStream_t st);
// Number of triangles whose three vertices are all in group 0 (static);
// the tile order puts them first.  Synchronises `st`.
hipError_t count_static(const uint32_t* idx, uint32_t ntri, const uint32_t* vgroup,
                        uint32_t* n_static, hipStream_t st);
// soup[3 t + k] = v[idx[3 t + k]] for the slots t < n
hipError_t launch_soup(const uint32_t* idx, const float4* v, uint32_t n, float4* soup,
                       hipStream_t st);

// The no-allocation cast's work memory: a static device array of
// NOALLOC_SCRATCH_BYTES, one per device.  noalloc_scratch_address gives its
// device address on the current device (call it once per device, with that
// device current); launch_put copies a small host record (a multiple of 4
// bytes) to device memory through kernel arguments, allocating nothing.
constexpr size_t NOALLOC_SCRATCH_BYTES = GRCA_NOALLOC_SCRATCH_BYTES;
constexpr uint32_t PUT_BLOB_WORDS = 1000;
hipError_t noalloc_scratch_address(void** out);
hipError_t launch_put(void* dst, const void* src, size_t bytes, hipStream_t st);
hipError_t launch_fill(uint32_t* a, uint32_t n, uint32_t v, hipStream_t st);

}  // namespace grca

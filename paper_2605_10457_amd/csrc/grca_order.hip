// grca_order.hip -- tile order of a scene's triangles.
//
// The bounds pass takes triangles 64 at a time and first tests the tile's
// bounding sphere against every sensor (group culling); a tile can only be
// culled when its triangles are close together.  Scenes arrive in any
// order (grids row by row, meshes as authored), so the scene's index
// buffer is stored in Morton order of triangle centroids, within each
// dynamic group (the static geometry, each rigid instance, each deforming
// range: a group moves as one piece, so its tiles stay compact when posed).
// `orig` maps each stored slot back to the caller's triangle id, which is
// what outputs and the closest-hit tie-break use.
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>
#include <algorithm>
#include <stdint.h>

#include "grca_launch.hpp"

namespace grca {

namespace {

__device__ inline int ordered_int(float f) {
  const int i = __float_as_int(f);
  return i >= 0 ? i : i ^ 0x7FFFFFFF;
}
__device__ inline float ordered_float(int i) { return __int_as_float(i >= 0 ? i : i ^ 0x7FFFFFFF); }

// box[0..2] = min x, y, z and box[3..5] = max, as order-preserving ints
__global__ void bbox_kernel(const float4* __restrict__ vtx, uint32_t nv, int* __restrict__ box) {
  float mn[3] = {3.0e38f, 3.0e38f, 3.0e38f}, mx[3] = {-3.0e38f, -3.0e38f, -3.0e38f};
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += gridDim.x * blockDim.x) {
    const float4 p = vtx[i];
    const float v[3] = {p.x, p.y, p.z};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      mn[k] = fminf(mn[k], v[k]);
      mx[k] = fmaxf(mx[k], v[k]);
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    for (int o = 32; o >= 1; o >>= 1) {
      mn[k] = fminf(mn[k], __shfl_xor(mn[k], o, 64));
      mx[k] = fmaxf(mx[k], __shfl_xor(mx[k], o, 64));
    }
  }
  if ((threadIdx.x & 63u) == 0u) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      atomicMin(box + k, ordered_int(mn[k]));
      atomicMax(box + 3 + k, ordered_int(mx[k]));
    }
  }
}

__global__ void init_box_kernel(int* box) {
  if (threadIdx.x < 3) box[threadIdx.x] = 0x7FFFFFFF;
  else if (threadIdx.x < 6) box[threadIdx.x] = (int)0x80000000;
}

__global__ void fill_kernel(uint32_t* __restrict__ a, uint32_t n, uint32_t v) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__device__ inline uint32_t spread10(uint32_t v) {  // 10 bits to every third bit
  v &= 0x3FFu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// key = dynamic group << 32 | 30-bit Morton code of the centroid
__global__ void order_keys_kernel(const uint32_t* __restrict__ idx, uint32_t ntri,
                                  const float4* __restrict__ v, const uint32_t* __restrict__ vgroup,
                                  const int* __restrict__ box,
                                  unsigned long long* __restrict__ keys,
                                  uint32_t* __restrict__ slots) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntri) return;
  const uint32_t i0 = idx[3ull * t], i1 = idx[3ull * t + 1], i2 = idx[3ull * t + 2];
  const float4 p0 = v[i0], p1 = v[i1], p2 = v[i2];
  const float c[3] = {(p0.x + p1.x + p2.x) * (1.0f / 3.0f), (p0.y + p1.y + p2.y) * (1.0f / 3.0f),
                      (p0.z + p1.z + p2.z) * (1.0f / 3.0f)};
  uint32_t code = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float lo = ordered_float(box[k]), hi = ordered_float(box[3 + k]);
    const float span = hi - lo;
    float q = span > 0.0f ? (c[k] - lo) / span * 1023.0f : 0.0f;
    q = fminf(fmaxf(q, 0.0f), 1023.0f);
    code |= spread10((uint32_t)q) << k;
  }
  // the largest group of the three vertices: a triangle touching a dynamic
  // vertex sorts after every all-static one
  const uint32_t g = max(vgroup[i0], max(vgroup[i1], vgroup[i2]));
  keys[t] = ((unsigned long long)g << 32) | code;
  slots[t] = t;
}

__global__ void order_gather_kernel(const uint32_t* __restrict__ idx_in,
                                    const uint32_t* __restrict__ orig_in,
                                    const uint32_t* __restrict__ perm, uint32_t ntri,
                                    uint32_t* __restrict__ idx_out,
                                    uint32_t* __restrict__ orig_out) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ntri) return;
  const uint32_t t = perm[k];
  idx_out[3ull * k] = idx_in[3ull * t];
  idx_out[3ull * k + 1] = idx_in[3ull * t + 1];
  idx_out[3ull * k + 2] = idx_in[3ull * t + 2];
  orig_out[k] = orig_in[t];
}

// Triangles whose three vertices are all static (group 0), counted with one
// atomic per wave.
// Grid-stride count, one atomic per wave at the end: the waves of a
// one-per-triangle grid (344k on 22M triangles) had queued on the one
// counter for 3 ms.
__global__ void count_static_kernel(const uint32_t* __restrict__ idx, uint32_t ntri,
                                    const uint32_t* __restrict__ vgroup,
                                    uint32_t* __restrict__ out) {
  uint32_t c = 0;
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < ntri; t += gridDim.x * blockDim.x)
    c += (vgroup[idx[3ull * t]] | vgroup[idx[3ull * t + 1]] | vgroup[idx[3ull * t + 2]]) == 0u;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63u) == 0u && c) atomicAdd(out, c);
}

// The vertex records of slots [0, n): soup[3 t + k] = v[idx[3 t + k]].
__global__ void soup_kernel(const uint32_t* __restrict__ idx, const float4* __restrict__ v,
                            uint32_t n, float4* __restrict__ soup) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 3ull * n) soup[i] = v[idx[i]];
}

__global__ void iota_kernel(uint32_t* __restrict__ a, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = i;
}

inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

}  // namespace

hipError_t launch_iota(uint32_t* a, uint32_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(iota_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, a, n);
  return hipGetLastError();
}

hipError_t launch_fill(uint32_t* a, uint32_t n, uint32_t v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, a, n, v);
  return hipGetLastError();
}

hipError_t count_static(const uint32_t* idx, uint32_t ntri, const uint32_t* vgroup,
                        uint32_t* n_static, hipStream_t st) {
  *n_static = 0;
  if (ntri == 0) return hipSuccess;
  uint32_t* d = nullptr;
  hipError_t e = hipMalloc(&d, sizeof(uint32_t));
  if (e != hipSuccess) return e;
  if ((e = hipMemsetAsync(d, 0, sizeof(uint32_t), st)) == hipSuccess) {
    hipLaunchKernelGGL(count_static_kernel, dim3((uint32_t)std::min<uint64_t>(cdiv(ntri, 256), 2048)),
                       dim3(256), 0, st, idx, ntri, vgroup, d);
    if ((e = hipGetLastError()) == hipSuccess)
      e = hipMemcpyAsync(n_static, d, sizeof(uint32_t), hipMemcpyDeviceToHost, st);
  }
  const hipError_t e2 = hipStreamSynchronize(st);
  (void)hipFree(d);
  return e != hipSuccess ? e : e2;
}

hipError_t launch_soup(const uint32_t* idx, const float4* v, uint32_t n, float4* soup,
                       hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(soup_kernel, dim3(cdiv(3ull * n, 256)), dim3(256), 0, st, idx, v, n, soup);
  return hipGetLastError();
}

hipError_t order_triangles(uint32_t* idx, uint32_t* orig, uint32_t ntri, const float4* v,
                           uint32_t nv, const uint32_t* vgroup, hipStream_t st) {
  if (ntri < 2 || nv == 0) return hipSuccess;
  hipError_t e = hipSuccess;
  int* box = nullptr;
  unsigned long long *k_in = nullptr, *k_out = nullptr;
  uint32_t *s_in = nullptr, *s_out = nullptr, *idx_new = nullptr, *orig_new = nullptr;
  void* temp = nullptr;
  size_t temp_bytes = 0;
  auto done = [&](hipError_t r) {
    (void)hipStreamSynchronize(st);
    if (box) (void)hipFree(box);
    if (k_in) (void)hipFree(k_in);
    if (k_out) (void)hipFree(k_out);
    if (s_in) (void)hipFree(s_in);
    if (s_out) (void)hipFree(s_out);
    if (idx_new) (void)hipFree(idx_new);
    if (orig_new) (void)hipFree(orig_new);
    if (temp) (void)hipFree(temp);
    return r;
  };
  if ((e = hipMalloc(&box, 6 * sizeof(int))) != hipSuccess) return done(e);
  if ((e = hipMalloc(&k_in, ntri * sizeof(unsigned long long))) != hipSuccess) return done(e);
  if ((e = hipMalloc(&k_out, ntri * sizeof(unsigned long long))) != hipSuccess) return done(e);
  if ((e = hipMalloc(&s_in, ntri * sizeof(uint32_t))) != hipSuccess) return done(e);
  if ((e = hipMalloc(&s_out, ntri * sizeof(uint32_t))) != hipSuccess) return done(e);
  if ((e = hipMalloc(&idx_new, 3ull * ntri * sizeof(uint32_t))) != hipSuccess) return done(e);
  if ((e = hipMalloc(&orig_new, ntri * sizeof(uint32_t))) != hipSuccess) return done(e);
  hipLaunchKernelGGL(init_box_kernel, dim3(1), dim3(64), 0, st, box);
  hipLaunchKernelGGL(bbox_kernel, dim3(std::min<uint32_t>(cdiv(nv, 256), 1024u)), dim3(256), 0,
                     st, v, nv, box);
  hipLaunchKernelGGL(order_keys_kernel, dim3(cdiv(ntri, 256)), dim3(256), 0, st, idx, ntri, v,
                     vgroup, box, k_in, s_in);
  if ((e = hipGetLastError()) != hipSuccess) return done(e);
  if ((e = hipcub::DeviceRadixSort::SortPairs(nullptr, temp_bytes, k_in, k_out, s_in, s_out,
                                              (int)ntri, 0, 64, st)) != hipSuccess)
    return done(e);
  if ((e = hipMalloc(&temp, temp_bytes)) != hipSuccess) return done(e);
  if ((e = hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, k_in, k_out, s_in, s_out,
                                              (int)ntri, 0, 64, st)) != hipSuccess)
    return done(e);
  hipLaunchKernelGGL(order_gather_kernel, dim3(cdiv(ntri, 256)), dim3(256), 0, st, idx, orig,
                     s_out, ntri, idx_new, orig_new);
  if ((e = hipGetLastError()) != hipSuccess) return done(e);
  if ((e = hipMemcpyAsync(idx, idx_new, 12ull * ntri, hipMemcpyDeviceToDevice, st)) != hipSuccess)
    return done(e);
  if ((e = hipMemcpyAsync(orig, orig_new, 4ull * ntri, hipMemcpyDeviceToDevice, st)) != hipSuccess)
    return done(e);
  return done(hipSuccess);
}

}  // namespace grca

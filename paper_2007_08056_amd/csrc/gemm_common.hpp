// Device helpers shared by the sector-product kernels (gemm.hip, gemm_bf16x3.hip):
// MFMA operand vector types, the XCD-aware tile order of one-workgroup-per-tile
// launches, global-to-LDS loads and the vector-memory wait.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace symt {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// Tile order of one-workgroup-per-tile launches: within each Q, groups of
// kGroupM M-panels, column by column, so the workgroups in flight on an XCD
// (a contiguous run of tiles, see xcd_remap) share A panels and B panels in L2.
constexpr int kGroupM = 8;
__device__ __forceinline__ void tile_coords(int64_t tile, int tiles_m, int tiles_n, int64_t& q, int& tm,
                                            int& tn, int group_m = kGroupM) {
  const int64_t per_q = static_cast<int64_t>(tiles_m) * tiles_n;
  q = tile / per_q;
  const int64_t t = tile - q * per_q;
  const int64_t group_tiles = static_cast<int64_t>(group_m) * tiles_n;
  const int64_t g = t / group_tiles;
  const int first_m = static_cast<int>(g * group_m);
  const int gm = min(tiles_m - first_m, group_m);
  const int r = static_cast<int>(t - g * group_tiles);
  tm = first_m + r % gm;
  tn = r / gm;
}

// Workgroups are dispatched round-robin over the 8 XCDs: remap their ids so
// that each XCD receives a contiguous run of tiles.
__device__ __forceinline__ int64_t xcd_remap(int64_t wg, int64_t n) {
  const int64_t per = n / 8;
  if (wg >= per * 8) return wg;
  return (wg % 8) * per + wg / 8;
}

template <typename T, int V>
struct alignas(sizeof(T) * V) VecT {
  T v[V];
};

// One 16-byte global load per lane straight into LDS (global_load_lds_dwordx4):
// lane i of the wave writes bytes [16 i, 16 i + 16) after the wave-uniform LDS base.
typedef __attribute__((address_space(1))) void* gptr_t;
typedef __attribute__((address_space(3))) void* lptr_t;
__device__ __forceinline__ void lds_dma16(const void* g, void* lds) {
  __builtin_amdgcn_global_load_lds((gptr_t)(g), (lptr_t)(lds), 16, 0, 0);
}

// s_waitcnt with vmcnt <= n and the other counters untouched (gfx9 encoding).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

}  // namespace
}  // namespace symt

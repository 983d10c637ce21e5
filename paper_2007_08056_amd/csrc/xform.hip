// Reduced-form transforms of the irrep-alignment method (Alg. 2: the step that
// forms the aligned operands, and its final step for the output).
//
// The aligned form of an operand and its standard reduced form hold the same
// blocks in a different arrangement: each aligned block (Q, stored row
// sectors, stored column sectors) is exactly one stored block of the standard
// form, because the generalized Kronecker deltas fix the two implicit sectors
// from Q.  So the transform is a block permutation plus one fixed permutation
// of the in-block indices -- constant work per element, the structured route
// the paper contrasts with dense delta contractions.  Each workgroup works
// inside one block; the block's two base offsets are computed once per
// workgroup from the group arithmetic.  Inside the block either
//   * copy mode: one run of elements is contiguous in both layouts; every
//     thread moves 16-byte vectors along it, rows indexed through LDS, or
//   * transpose mode: the source- and destination-contiguous dims differ;
//     a 64 x 64 tile is read into LDS along index A (the source-fastest dims,
//     merged until 64 elements) and written along index B (the
//     destination-fastest of the rest), so in-block dims as small as 2 still
//     fill the tile.
// Element conversions (f64 <-> f32, f32 -> bf16 hi/lo pair) are fused.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "bf16_split.hpp"
#include "plan.hpp"
#include "xform_index.hpp"

namespace symt {

namespace {

template <typename T, int V>
struct alignas(sizeof(T) * V) VecT {
  T v[V];
};

// OUT: 0 -> f64, 1 -> f32, 2 -> bf16 hi plane at off, lo plane at off + plane;
// il: the planes interleaved by 32-deep K-steps (hi at 2 off - off % 32; the V
// elements of one store stay inside one K-step).
template <int OUT, int V>
__device__ __forceinline__ void store_vec(void* dst, int64_t off, int64_t plane, const double (&x)[V], int il = 0) {
  if constexpr (OUT == 0) {
    VecT<double, V> o;
#pragma unroll
    for (int i = 0; i < V; ++i) o.v[i] = x[i];
    *reinterpret_cast<VecT<double, V>*>(static_cast<double*>(dst) + off) = o;
  } else if constexpr (OUT == 1) {
    VecT<float, V> o;
#pragma unroll
    for (int i = 0; i < V; ++i) o.v[i] = static_cast<float>(x[i]);
    *reinterpret_cast<VecT<float, V>*>(static_cast<float*>(dst) + off) = o;
  } else {
    VecT<uint16_t, V> h, l;
#pragma unroll
    for (int i = 0; i < V; ++i) bf16_split(x[i], h.v[i], l.v[i]);
    uint16_t* d = static_cast<uint16_t*>(dst);
    if (il) off = 2 * off - (off & 31);
    *reinterpret_cast<VecT<uint16_t, V>*>(d + off) = h;
    *reinterpret_cast<VecT<uint16_t, V>*>(d + off + plane) = l;
  }
}

template <typename Tin, int OUT, int V>
__global__ __launch_bounds__(256) void k_xform_copy(const Tin* __restrict__ src,
                                                    void* __restrict__ dst, const XformParams p) {
  constexpr int kRows = 1024;                    // rows whose offsets sit in LDS at once
  __shared__ int64_t soff[kRows];
  __shared__ int64_t doff[kRows];
  // (the launch has at most 2^31 - 1 workgroups: 32-bit workgroup arithmetic)
  const int wg = static_cast<int>(blockIdx.x);
  const int tpb = static_cast<int>(p.tiles_per_block), rt = static_cast<int>(p.run_tiles);
  const int blk = wg / tpb;
  const int tile = wg - blk * tpb;
  const int row_tile = tile / rt;
  const int64_t c_begin = static_cast<int64_t>(tile - row_tile * rt) * p.run_chunk;
  const int64_t c_end = c_begin + p.run_chunk < p.run_len ? c_begin + p.run_chunk : p.run_len;
  int64_t sb, ab;
  // a block that does not exist (subgroup modes): its aligned block is zero,
  // and there is nothing to write into the (cleared) standard form
  const bool live = block_bases(p, blk, sb, ab);
  if (!live && !p.to_aligned) return;
  const int64_t src_base = p.to_aligned ? sb : ab;
  const int64_t dst_base = p.to_aligned ? ab : sb;
  // this workgroup's rows [r_begin, r_end), moved kRows at a time (their offsets in LDS)
  const int64_t r_begin = row_tile * p.rows_per_tile;
  const int64_t r_end = r_begin + p.rows_per_tile < p.rows ? r_begin + p.rows_per_tile : p.rows;
  const int lane = threadIdx.x & (p.lanes_per_row - 1);
  const int sub = threadIdx.x >> p.lanes_log2;
  const int rpp = blockDim.x >> p.lanes_log2;
  const int64_t step = static_cast<int64_t>(p.lanes_per_row) * V;
  for (int64_t r0 = r_begin; r0 < r_end; r0 += kRows) {
  const int nr = static_cast<int>(r_end - r0 < kRows ? r_end - r0 : kRows);
  if (r0 > r_begin) __syncthreads();             // the previous rows' offsets are no longer read
  for (int r = threadIdx.x; r < nr; r += blockDim.x) {
    int64_t so = 0, dof = 0;
    if (p.rows <= INT32_MAX) batch_offsets<int32_t>(p, static_cast<int32_t>(r0 + r), so, dof);
    else batch_offsets<int64_t>(p, r0 + r, so, dof);
    soff[r] = src_base + so;
    doff[r] = dst_base + dof;
  }
  __syncthreads();
  // Four loads go out before their stores (a load waits for nothing but its
  // own data): four rows at a time where each lane holds at most one vector of
  // a row, else four vectors of one row at a time.
  auto load = [&](int64_t s0, int64_t c, double (&x)[V]) {
    if constexpr (V == 1) {
      x[0] = live ? static_cast<double>(src[s0 + c * p.run_ss]) : 0.0;
    } else {
      if (live) {
        const VecT<Tin, V> in = *reinterpret_cast<const VecT<Tin, V>*>(src + s0 + c);
#pragma unroll
        for (int i = 0; i < V; ++i) x[i] = static_cast<double>(in.v[i]);
      } else {
#pragma unroll
        for (int i = 0; i < V; ++i) x[i] = 0.0;
      }
    }
  };
  auto store = [&](int64_t d0, int64_t c, const double (&x)[V]) {
    store_vec<OUT, V>(dst, d0 + (V == 1 ? c * p.run_ds : c), p.plane, x, p.il);
  };
  constexpr int U = 4;
  const int64_t c0 = c_begin + static_cast<int64_t>(lane) * V;
  if (c_end - c_begin <= step) {
    if (c0 < c_end) {
      for (int r = sub; r < nr; r += U * rpp) {
        double x[U][V];
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (r + u * rpp < nr) load(soff[r + u * rpp], c0, x[u]);
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (r + u * rpp < nr) store(doff[r + u * rpp], c0, x[u]);
      }
    }
  } else {
    for (int r = sub; r < nr; r += rpp) {
      const int64_t s0 = soff[r], d0 = doff[r];
      for (int64_t c = c0; c < c_end; c += U * step) {
        double x[U][V];
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (c + u * step < c_end) load(s0, c + u * step, x[u]);
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (c + u * step < c_end) store(d0, c + u * step, x[u]);
      }
    }
  }
  }
}

// Offsets (source, destination) of entry i of a mixed-radix tile index (I: the
// index type, 32-bit where the tile's index range fits).
template <typename I>
__device__ __forceinline__ void tile_offsets(I i, int n, const int64_t* size, const int64_t* ss,
                                             const int64_t* ds, int64_t& so, int64_t& dof) {
  so = 0;
  dof = 0;
  for (int k = 0; k < n; ++k) {
    const I sz = static_cast<I>(size[k]);
    const I q = i / sz;
    const I c = i - q * sz;
    i = q;
    so += static_cast<int64_t>(c) * ss[k];
    dof += static_cast<int64_t>(c) * ds[k];
  }
}

template <typename Tin, int OUT>
__global__ __launch_bounds__(256) void k_xform_transpose(const Tin* __restrict__ src,
                                                         void* __restrict__ dst,
                                                         const XformParams p) {
  __shared__ double tile[64][65];
  __shared__ int64_t a_src[64], a_dst[64], b_src[64], b_dst[64];
  __shared__ int perm[64];                        // tr_write: A elements in destination order
  // (the launch has at most 2^31 - 1 workgroups: 32-bit workgroup arithmetic)
  const int wg = static_cast<int>(blockIdx.x);
  const int tpb = static_cast<int>(p.tiles_per_block);
  const int blk = wg / tpb;
  int rem = wg - blk * tpb;
  const int tb = rem % p.tiles_t;
  rem /= p.tiles_t;
  const int ta = rem % p.tiles_run;
  const int row = rem / p.tiles_run;
  int64_t sb, ab;
  const bool live = block_bases(p, blk, sb, ab);
  if (!live && !p.to_aligned) return;             // as in k_xform_copy
  int64_t so = p.to_aligned ? sb : ab;
  int64_t dof = p.to_aligned ? ab : sb;
  batch_offsets<int32_t>(p, row, so, dof);
  const int64_t a0 = static_cast<int64_t>(ta) * 64, b0 = static_cast<int64_t>(tb) * 64;
  const int na = static_cast<int>(p.run_len - a0 < 64 ? p.run_len - a0 : 64);
  const int nb = static_cast<int>(p.t_len - b0 < 64 ? p.t_len - b0 : 64);
  const int t = threadIdx.x;
  if (t < 64) {
    if (t < na) {
      if (p.run_len <= INT32_MAX) tile_offsets<int32_t>(static_cast<int32_t>(a0 + t), p.na, p.asize, p.ass, p.ads, a_src[t], a_dst[t]);
      else tile_offsets<int64_t>(a0 + t, p.na, p.asize, p.ass, p.ads, a_src[t], a_dst[t]);
    }
  } else if (t < 128) {
    const int u = t - 64;
    if (u < nb) {
      if (p.t_len <= INT32_MAX) tile_offsets<int32_t>(static_cast<int32_t>(b0 + u), p.nb, p.tsize, p.tss, p.tds, b_src[u], b_dst[u]);
      else tile_offsets<int64_t>(b0 + u, p.nb, p.tsize, p.tss, p.tds, b_src[u], b_dst[u]);
    }
  }
  __syncthreads();
  const int x = t & 63;
  const int y = t >> 6;
  if (p.tr_write && t < na) {
    // rank of this A element by destination offset (ties by index): a permutation
    int rk = 0;
    for (int u = 0; u < na; ++u) rk += a_dst[u] < a_dst[t] || (a_dst[u] == a_dst[t] && u < t);
    perm[rk] = t;
  }
  if (x < na) {
    // all sixteen of this thread's loads go out before the first LDS write
    const int64_t sx = so + a_src[x];
    double v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int j = y + 4 * k;
      v[k] = live && j < nb ? static_cast<double>(src[sx + b_src[j]]) : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k)
      if (y + 4 * k < nb) tile[y + 4 * k][x] = v[k];
  }
  __syncthreads();
  if (p.tr_write) {
    // lanes along the A side in destination order, B rows in turn
    if (x < na) {
      const int ae = perm[x];
      const int64_t da = dof + a_dst[ae];
      for (int j = y; j < nb; j += 4) {
        double v[1] = {tile[j][ae]};
        store_vec<OUT, 1>(dst, da + b_dst[j], p.plane, v, p.il);
      }
    }
  } else if (x < nb) {
    const int64_t dx = dof + b_dst[x];
    for (int j = y; j < na; j += 4) {
      double v[1] = {tile[x][j]};
      store_vec<OUT, 1>(dst, dx + a_dst[j], p.plane, v, p.il);
    }
  }
}

template <typename Tin, int OUT>
hipError_t launch_typed(const XformParams& p, const void* src, void* dst, hipStream_t stream) {
  const int64_t nwg = p.nblocks * p.tiles_per_block;
  const dim3 grid(static_cast<unsigned>(nwg)), block(256);
  const Tin* s = static_cast<const Tin*>(src);
  if (p.mode == 1) {
    hipLaunchKernelGGL((k_xform_transpose<Tin, OUT>), grid, block, 0, stream, s, dst, p);
  } else if (p.vec == 4) {
    if constexpr (sizeof(Tin) * 4 <= 16 && (OUT != 0))
      hipLaunchKernelGGL((k_xform_copy<Tin, OUT, 4>), grid, block, 0, stream, s, dst, p);
    else
      hipLaunchKernelGGL((k_xform_copy<Tin, OUT, 1>), grid, block, 0, stream, s, dst, p);
  } else if (p.vec == 2) {
    hipLaunchKernelGGL((k_xform_copy<Tin, OUT, 2>), grid, block, 0, stream, s, dst, p);
  } else {
    hipLaunchKernelGGL((k_xform_copy<Tin, OUT, 1>), grid, block, 0, stream, s, dst, p);
  }
  return hipGetLastError();
}

// (I: the index type, 32-bit when every table's entry count fits)
template <typename I>
__global__ __launch_bounds__(256) void k_offsets(const OffsetBatch b) {
  const I total = static_cast<I>(b.n > 0 ? b.end[b.n - 1] : 0);
  const I stride = static_cast<I>(gridDim.x) * blockDim.x;
  for (I i = static_cast<I>(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += stride) {
    int t = 0;
    while (i >= b.end[t]) ++t;
    const I j = i - static_cast<I>(t > 0 ? b.end[t - 1] : 0);
    const OffsetParams& p = b.t[t];
    const int q = static_cast<int>(j / static_cast<I>(p.count));
    b.out[t][j] = table_entry(p, q, j - static_cast<I>(q) * static_cast<I>(p.count));
  }
}

// Odd rows of a complex V_al in the real representation of C: in every slice,
// real row 2k + 1 holds (-im, re) of the (re, im) pairs in row 2k.  One thread
// per pair; `rows` complex rows and `pairs` complex columns per slice.
template <typename T>
__global__ __launch_bounds__(256) void k_cplx_rows(T* __restrict__ v, int64_t slices, int64_t rows,
                                                   int64_t pairs) {
  const int64_t total = slices * rows * pairs;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int64_t c = i % pairs;
    const int64_t r = i / pairs;                  // slice * rows + row
    T* even = v + (2 * r) * (2 * pairs) + 2 * c;
    const T re = even[0], im = even[1];
    even[2 * pairs] = -im;
    even[2 * pairs + 1] = re;
  }
}

// The same for split-bf16 V planes, stored K fastest ([slice][real column][K
// pitch kp]): real row 2k + 1 of column pair (2n, 2n + 1) holds (-im, re) of
// row 2k, in the hi plane at v and the lo plane at v + plane.  Negation only
// flips the sign bit, so the pair is the split of (-im, re) exactly.
__global__ __launch_bounds__(256) void k_cplx_rows_planes(uint16_t* __restrict__ v, int64_t plane, int64_t slices,
                                                          int64_t rows, int64_t pairs, int64_t kp) {
  const int64_t total = slices * pairs * rows;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int64_t k = i % rows;
    const int64_t t = i / rows;
    const int64_t n = t % pairs;
    const int64_t sl = t / pairs;
    const int64_t re = (sl * 2 * pairs + 2 * n) * kp + 2 * k;    // (2k, 2n)
    const int64_t im = re + kp;                                   // (2k, 2n + 1)
#pragma unroll
    for (int pl = 0; pl < 2; ++pl) {
      uint16_t* b = v + pl * plane;
      const uint16_t r = b[re], m = b[im];
      b[re + 1] = static_cast<uint16_t>(m ^ 0x8000u);              // (2k + 1, 2n) = -im
      b[im + 1] = r;                                              // (2k + 1, 2n + 1) = re
    }
  }
}

// A few KB of host data (charge tables) written into device memory from kernel
// arguments: stream-ordered, with no host buffer that must outlive the call.
struct I32Chunk {
  int32_t v[512];
};

__global__ __launch_bounds__(256) void k_put_i32(int32_t* __restrict__ dst, int n, const I32Chunk c) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = c.v[i];
}

}  // namespace

int launch_put_i32(int32_t* dst, const int32_t* src, int64_t n, hipStream_t stream, std::string* err) {
  for (int64_t o = 0; o < n; o += 512) {
    I32Chunk c;
    const int k = static_cast<int>(n - o < 512 ? n - o : 512);
    for (int i = 0; i < k; ++i) c.v[i] = src[o + i];
    hipLaunchKernelGGL(k_put_i32, dim3(1), dim3(256), 0, stream, dst + o, k, c);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      if (err) *err = std::string("charge table upload: ") + hipGetErrorString(e);
      return SYMT_EHIP;
    }
  }
  return SYMT_OK;
}

int launch_cplx_rows(void* v, bool f64, int64_t slices, int64_t rows, int64_t pairs, hipStream_t stream,
                     std::string* err) {
  const int64_t total = slices * rows * pairs;
  if (total == 0) return SYMT_OK;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (f64)
    hipLaunchKernelGGL(k_cplx_rows<double>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream,
                       static_cast<double*>(v), slices, rows, pairs);
  else
    hipLaunchKernelGGL(k_cplx_rows<float>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream,
                       static_cast<float*>(v), slices, rows, pairs);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    if (err) *err = std::string("complex rows launch: ") + hipGetErrorString(e);
    return SYMT_EHIP;
  }
  return SYMT_OK;
}

int launch_cplx_rows_planes(void* v, int64_t plane, int64_t slices, int64_t rows, int64_t pairs, int64_t kp,
                            hipStream_t stream, std::string* err) {
  const int64_t total = slices * rows * pairs;
  if (total == 0) return SYMT_OK;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_cplx_rows_planes, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream,
                     static_cast<uint16_t*>(v), plane, slices, rows, pairs, kp);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    if (err) *err = std::string("complex rows launch: ") + hipGetErrorString(e);
    return SYMT_EHIP;
  }
  return SYMT_OK;
}

__global__ __launch_bounds__(256) void k_zero_u32(uint32_t* __restrict__ p, int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0u;
}

// Clears `bytes` (a multiple of 4) at a 4-byte aligned device address; a kernel
// rather than a memset node, so that captured streams replay it reliably.
int launch_zero(void* ptr, size_t bytes, hipStream_t stream, std::string* err) {
  const int64_t n = static_cast<int64_t>(bytes / 4);
  if (n == 0) return SYMT_OK;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_zero_u32, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream,
                     static_cast<uint32_t*>(ptr), n);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    if (err) *err = std::string("clear launch: ") + hipGetErrorString(e);
    return SYMT_EHIP;
  }
  return SYMT_OK;
}

// Every table of the batch in one launch.
int launch_offsets(const OffsetBatch& batch, hipStream_t stream, std::string* err) {
  const int64_t total = batch.n > 0 ? batch.end[batch.n - 1] : 0;
  if (total == 0) return SYMT_OK;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (total + static_cast<int64_t>(blocks) * 256 <= INT32_MAX)
    hipLaunchKernelGGL(k_offsets<int32_t>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, batch);
  else
    hipLaunchKernelGGL(k_offsets<int64_t>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, batch);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    if (err) *err = std::string("offset table launch: ") + hipGetErrorString(e);
    return SYMT_EHIP;
  }
  return SYMT_OK;
}

// in_f64: source elements are binary64 (else binary32); out: 0 f64, 1 f32, 2 bf16 split.
int launch_xform(const XformParams& p, bool in_f64, int out, const void* src, void* dst,
                 hipStream_t stream, std::string* err) {
  const int64_t nwg = p.nblocks * p.tiles_per_block;
  if (nwg == 0) return SYMT_OK;
  if (nwg > INT32_MAX) {
    if (err) *err = "transform needs more than 2^31-1 workgroups";
    return SYMT_EUNSUPPORTED;
  }
  hipError_t e;
  if (in_f64) {
    e = out == 0 ? launch_typed<double, 0>(p, src, dst, stream)
        : out == 1 ? launch_typed<double, 1>(p, src, dst, stream)
                   : launch_typed<double, 2>(p, src, dst, stream);
  } else {
    e = out == 0 ? launch_typed<float, 0>(p, src, dst, stream)
        : out == 1 ? launch_typed<float, 1>(p, src, dst, stream)
                   : launch_typed<float, 2>(p, src, dst, stream);
  }
  if (e != hipSuccess) {
    if (err) *err = std::string("transform launch: ") + hipGetErrorString(e);
    return SYMT_EHIP;
  }
  return SYMT_OK;
}

}  // namespace symt

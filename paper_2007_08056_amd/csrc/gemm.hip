// Sector-batched dense product of the aligned forms (Alg. 2's product step;
// the einsum "AQL,LQJ->AQJ" of Sec. 2.1): for every auxiliary sector Q,
// C[Q] (M x N) = A[Q] (M x K) * B[Q] (K x N), all slices the same shape.
//
// gfx950 MFMA kernels, one workgroup per (Q, BM x BN) output tile:
//   * f64: v_mfma_f64_16x16x4_f64, f32: v_mfma_f32_16x16x4_f32.  A and B
//     tiles are staged through LDS in double buffers (A as [m][k], B as
//     [k][n], both padded), one barrier per K step.
//   * split-bf16: A = Ahi + Alo and B = Bhi + Blo (bf16 planes, B stored
//     [Q][N][K]); v_mfma_f32_16x16x32_bf16 forms Ahi*Bhi in one binary32
//     accumulator and Ahi*Blo + Alo*Bhi in a second; the epilogue adds the two
//     in binary64 and stores binary64.
// Workgroups are dispatched round-robin over the 8 XCDs; the tile order is
// remapped so that each XCD receives a contiguous run of tiles (the N tiles
// of one M panel land on the same XCD and share its L2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <string>
#include <type_traits>

#include "bf16_split.hpp"
#include "gemm_common.hpp"
#include "plan.hpp"
#include "sk_index.hpp"

namespace symt {

namespace {

template <typename T>
struct Mfma;
// Accumulator layouts (lane l, item r, column l % 16): the f64 16x16x4 form
// holds row l/16 + 4r, the f32 16x16x4 and bf16 16x16x32 forms row 4(l/16) + r.
template <>
struct Mfma<double> {
  using Acc = d4;
  static __device__ __forceinline__ Acc run(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct Mfma<float> {
  using Acc = f4;
  static __device__ __forceinline__ Acc run(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// ---------------------------------------------------------------------------
// f64 / f32: C = A B, A [Q][M][K], B [Q][K][N], C [Q][M][N], row-major.
// V: elements per global vector access (16 bytes, or 1 when K or N is odd).
// ---------------------------------------------------------------------------
// Fused forms (FA / FC): A is read straight from U's standard reduced form,
// element (q, m, k) at ra[q*M + m] + ca[q*K + k], and C is written straight
// into W's standard reduced form at rc[q*M + m] + cc[q*N + n] (separable offset
// tables).  FA needs every K-step to be contiguous in U (BK-aligned steps of K,
// or steps of each run with krun below).
// With FA and rb given, B is V's standard form: row k0 + r of a K-step at
// rb[q*K + k0] + r * ldb, column n at cb[q*N + n] (every K-step inside one affine
// run of rows, every V-wide load inside one contiguous run of columns).
// krun > 0: K is K / krun runs of krun indices, and each run is stepped on its
// own (ceil(krun / BK) steps, the last one masked past the run's end), so a
// K-step never straddles two runs whatever krun is; krun = 0 steps K plainly.
// SPLIT: gridDim.x = ntiles * splits; workgroup (tile, s) multiplies the s-th of
// `splits` equal runs of K-steps and stores its partial tile in accumulator
// order at part + (tile * splits + s) * BM * BN; k_split_sum adds them.
// AT (with FA): A is loaded K-major, as B is: row k0 + r of a K-step at
// ca[q*K + k0 + r] (any layout of U's contracted modes), V-wide chunks of M at
// ra[q*M + m] (contiguous runs of U's other modes); the LDS tile is [k][m].
// ATK (with AT): U's other modes hold no such chunks but its contracted modes
// end in runs of V: lanes load V consecutive K indices of one row m
// (ra[q*M + m] + ca[q*K + k] .. + V - 1) and write them down the [k][m] tile.
template <typename T, int BM, int BN, int BK, int WM, int WN, int V, bool FA, bool FC, bool SPLIT = false,
          bool AT = false, bool ATK = false>
__global__ __launch_bounds__(64 * WM * WN) void k_gemm(const T* __restrict__ A,
                                                       const T* __restrict__ B,
                                                       T* __restrict__ C, int M, int N, int K,
                                                       int tiles_m, int tiles_n, int64_t ntiles,
                                                       const int64_t* __restrict__ ra,
                                                       const int64_t* __restrict__ ca,
                                                       const int64_t* __restrict__ rc,
                                                       const int64_t* __restrict__ cc,
                                                       T* __restrict__ part = nullptr, int splits = 1,
                                                       const int64_t* __restrict__ rb = nullptr,
                                                       const int64_t* __restrict__ cb = nullptr,
                                                       int64_t ldb = 0, int krun = 0) {
  constexpr int NT = 64 * WM * WN;
  constexpr int PAD = 16 / sizeof(T);
  // B rows: a fragment read touches 16 consecutive n at 4 consecutive k; pad each
  // row so that the 4 rows start 16 * sizeof(T) bytes apart modulo the 256-byte
  // bank cycle, which keeps the four 16-lane groups on disjoint banks.
  constexpr int ROWB = BN * static_cast<int>(sizeof(T));
  constexpr int SHIFT = 16 * static_cast<int>(sizeof(T));
  constexpr int PADB = ((SHIFT - ROWB % 256 + 256) % 256) / static_cast<int>(sizeof(T));
  constexpr int TM = BM / WM / 16;
  constexpr int TN = BN / WN / 16;
  static_assert(TM * WM * 16 == BM && TN * WN * 16 == BN, "tile shape");
  static_assert(BK % 4 == 0, "BK");
  constexpr int LA = (BM * BK / V + NT - 1) / NT;   // vector loads per thread, A tile
  constexpr int LB = (BK * BN / V + NT - 1) / NT;   // vector loads per thread, B tile
  using Acc = typename Mfma<T>::Acc;
  static_assert(!AT || FA, "A is loaded K-major from U's standard form only");
  // K-major A rows padded as B's are
  constexpr int PADA = ((SHIFT - (BM * static_cast<int>(sizeof(T))) % 256 + 256) % 256) /
                       static_cast<int>(sizeof(T));

  __shared__ T As[2][AT ? 1 : BM][AT ? 1 : BK + PAD];
  __shared__ T AsT[2][AT ? BK : 1][AT ? BM + PADA : 1];
  __shared__ T Bs[2][BK][BN + PADB];

  const int64_t tile = SPLIT ? static_cast<int64_t>(blockIdx.x) / splits : xcd_remap(blockIdx.x, ntiles);
  const int split = SPLIT ? static_cast<int>(blockIdx.x - tile * splits) : 0;
  int64_t q;
  int tm, tn;
  tile_coords(tile, tiles_m, tiles_n, q, tm, tn);
  const bool fb = FA && rb != nullptr;   // uniform: B read in place
  const T* Aq = A + (FA ? 0 : q * static_cast<int64_t>(M) * K);
  const T* Bq = B + (fb ? 0 : q * static_cast<int64_t>(K) * N);
  T* Cq = C + (FC ? 0 : q * static_cast<int64_t>(M) * N);
  const int m0 = tm * BM, n0 = tn * BN;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave / WN) * (BM / WM);
  const int wn0 = (wave % WN) * (BN / WN);

  // Fused A: the standard-form offset of each of this thread's tile rows (AT:
  // of the M chunk it loads in every K-step).
  static_assert(!ATK || (AT && BK % V == 0), "K vectors of A need K-major A and whole vectors per step");
  int64_t arow[LA];
#pragma unroll
  for (int i = 0; i < LA; ++i) {
    const int e = (tid + i * NT) * V;
    const int gr = m0 + (AT && !ATK ? e % BM : e / BK);
    arow[i] = (FA && e < BM * BK && gr < M) ? ra[q * M + gr] : static_cast<int64_t>(gr) * K;
  }

  // B: offset of each of this thread's tile positions, fixed across K-steps
  // (row r of the step, column gc), plus one row offset per K-step
  int64_t bpos[LB];
#pragma unroll
  for (int i = 0; i < LB; ++i) {
    const int e = (tid + i * NT) * V;
    const int r = e / BN, gc = n0 + e % BN;
    bpos[i] = fb ? static_cast<int64_t>(r) * ldb + (e < BK * BN && gc < N ? cb[q * N + gc] : 0)
                 : static_cast<int64_t>(r) * N + gc;
  }

  VecT<T, V> ra_[LA], rb_[LB];
  // K-step kt starts at k0 and holds kv valid indices (uniform)
  const int spr = krun > 0 ? (krun + BK - 1) / BK : 0;
  auto load_tiles = [&](int kt) {
    int k0, kv;
    if (krun > 0) {
      const int run = kt / spr, st = kt - run * spr;
      k0 = run * krun + st * BK;
      kv = min(BK, krun - st * BK);
    } else {
      k0 = kt * BK;
      kv = K - k0;
    }
    const int64_t acol = FA ? ca[q * K + k0] : k0;
    const int64_t brow = fb ? rb[q * K + k0] : static_cast<int64_t>(k0) * N;
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int e = (tid + i * NT) * V;              // element index inside the BM x BK tile
      if constexpr (ATK) {                           // row m, K vector c of the step
        const int m = e / BK, c = e % BK;
        if (e < BM * BK && m0 + m < M && c < kv)
          ra_[i] = *reinterpret_cast<const VecT<T, V>*>(Aq + ca[q * K + k0 + c] + arow[i]);
        else
#pragma unroll
          for (int j = 0; j < V; ++j) ra_[i].v[j] = T(0);
      } else if constexpr (AT) {                     // [k][m]: row r of the step, M chunk c
        const int r = e / BM, c = e % BM;
        if (e < BM * BK && m0 + c < M && r < kv)
          ra_[i] = *reinterpret_cast<const VecT<T, V>*>(Aq + ca[q * K + k0 + r] + arow[i]);
        else
#pragma unroll
          for (int j = 0; j < V; ++j) ra_[i].v[j] = T(0);
      } else {
        const int r = e / BK, c = e % BK;
        const int gr = m0 + r;
        if (e < BM * BK && gr < M && c < kv)
          ra_[i] = *reinterpret_cast<const VecT<T, V>*>(Aq + arow[i] + acol + c);
        else
#pragma unroll
          for (int j = 0; j < V; ++j) ra_[i].v[j] = T(0);
      }
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int e = (tid + i * NT) * V;              // element index inside the BK x BN tile
      const int r = e / BN, c = e % BN;
      const int gc = n0 + c;
      if (e < BK * BN && r < kv && gc < N)
        rb_[i] = *reinterpret_cast<const VecT<T, V>*>(Bq + brow + bpos[i]);
      else
#pragma unroll
        for (int j = 0; j < V; ++j) rb_[i].v[j] = T(0);
    }
  };
  auto store_tiles = [&](int buf) {
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int e = (tid + i * NT) * V;
      if constexpr (ATK) {
        if (e < BM * BK)
#pragma unroll
          for (int j = 0; j < V; ++j) AsT[buf][e % BK + j][e / BK] = ra_[i].v[j];
      } else if constexpr (AT) {
        if (e < BM * BK) *reinterpret_cast<VecT<T, V>*>(&AsT[buf][e / BM][e % BM]) = ra_[i];
      } else {
        if (e < BM * BK) *reinterpret_cast<VecT<T, V>*>(&As[buf][e / BK][e % BK]) = ra_[i];
      }
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int e = (tid + i * NT) * V;
      if (e < BK * BN) *reinterpret_cast<VecT<T, V>*>(&Bs[buf][e / BN][e % BN]) = rb_[i];
    }
  };

  Acc acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = Acc{};

  const int nk_all = krun > 0 ? K / krun * spr : (K + BK - 1) / BK;
  // this workgroup's K-steps [kt0, kt1): all of them, or its split's share
  const int per = SPLIT ? (nk_all + splits - 1) / splits : nk_all;
  const int kt0 = SPLIT ? min(nk_all, split * per) : 0;
  const int kt1 = SPLIT ? min(nk_all, kt0 + per) : nk_all;
  if (kt0 < kt1) {
    load_tiles(kt0);
    store_tiles(0);
  }
  __syncthreads();
  for (int kt = kt0; kt < kt1; ++kt) {
    const int buf = (kt - kt0) & 1;
    if (kt + 1 < kt1) load_tiles(kt + 1);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i)
        a[i] = AT ? AsT[buf][kk + (lane >> 4)][wm0 + i * 16 + (lane & 15)]
                  : As[buf][wm0 + i * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] = Bs[buf][kk + (lane >> 4)][wn0 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = Mfma<T>::run(a[i], b[j], acc[i][j]);
    }
    if (kt + 1 < kt1) store_tiles(buf ^ 1);
    __syncthreads();
  }

  if constexpr (SPLIT) {
    // partial tile in accumulator order: element ((wave*TM + i)*TN + j)*4 + r of lane l
    // at 64 * that + l, so these stores and k_split_sum's loads coalesce
    T* pw = part + (tile * splits + split) * static_cast<int64_t>(BM * BN) + wave * (TM * TN * 4 * 64) + lane;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) pw[((i * TN + j) * 4 + r) * 64] = acc[i][j][r];
    return;
  }
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int col = n0 + wn0 + j * 16 + (lane & 15);
    const int64_t ccol = (FC && col < N) ? cc[q * N + col] : col;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm0 + i * 16 + Mfma<T>::row(lane, r);
        if (row < M && col < N) {
          const int64_t crow = FC ? rc[q * M + row] : static_cast<int64_t>(row) * N;
          Cq[crow + ccol] = acc[i][j][r];
        }
      }
  }
}

// Sums the `splits` partial tiles of each tile in split order (so the result does
// not depend on scheduling) and writes the tile, as k_gemm's epilogue would.
// Workgroup (tile, chunk) sums one range of the tile's elements: each element
// starts from zero and adds its splits in order whatever the chunk count.
template <typename T, int BM, int BN, int WM, int WN, bool FC>
__global__ __launch_bounds__(64 * WM * WN) void k_split_sum(const T* __restrict__ part, T* __restrict__ C,
                                                            int M, int N, int tiles_m, int tiles_n, int splits,
                                                            const int64_t* __restrict__ rc,
                                                            const int64_t* __restrict__ cc) {
  constexpr int TM = BM / WM / 16, TN = BN / WN / 16;
  constexpr int E = BM * BN;
  constexpr int NT = 64 * WM * WN;
  constexpr int PER_WAVE = TM * TN * 4 * 64;
  const int64_t tile = blockIdx.x;
  int64_t q;
  int tm, tn;
  tile_coords(tile, tiles_m, tiles_n, q, tm, tn);
  T* Cq = C + (FC ? 0 : q * static_cast<int64_t>(M) * N);
  const T* pt = part + tile * splits * static_cast<int64_t>(E);
  // workgroup (tile, chunk): the chunk-th of gridDim.y equal ranges of the
  // tile's elements in accumulator order
  const int chunks = static_cast<int>(gridDim.y);
  const int per = (E + chunks - 1) / chunks;
  const int e0 = static_cast<int>(blockIdx.y) * per;
  const int e1 = min(E, e0 + per);
  for (int e = e0 + static_cast<int>(threadIdx.x); e < e1; e += NT) {
    // accumulator order: element ((w * TM + i) * TN + j) * 4 + r of lane l at 64 * that + l
    // (W's table entries requested before the partials are read)
    const int w = e / PER_WAVE;
    const int rem = e - w * PER_WAVE;
    const int lane = rem & 63;
    const int ijr = rem >> 6;
    const int r = ijr & 3;
    const int ij = ijr >> 2;
    const int i = ij / TN, j = ij - (ij / TN) * TN;
    const int row = tm * BM + (w / WN) * (BM / WM) + i * 16 + Mfma<T>::row(lane, r);
    const int col = tn * BN + (w % WN) * (BN / WN) + j * 16 + (lane & 15);
    const bool in = row < M && col < N;
    const int64_t crow = FC ? (in ? rc[q * M + row] : 0) : static_cast<int64_t>(row) * N;
    const int64_t ccol = FC ? (in ? cc[q * N + col] : 0) : col;
    T acc = T(0);
#pragma unroll 8
    for (int sp = 0; sp < splits; ++sp) acc += pt[static_cast<int64_t>(sp) * E + e];
    if (in) Cq[crow + ccol] = acc;
  }
}

// ---------------------------------------------------------------------------
// f64 / f32 with direct global->LDS loads (global_load_lds_dwordx4) into an
// S-stage LDS ring: tile k+S-1 streams into LDS while tile k is multiplied, so
// S-1 K-steps of latency are hidden without staging registers; one barrier per
// K-step.  A rows are 128 bytes (BK = 128 / sizeof(T)), 8 chunks of 16 bytes.
// Lane i of a wave load writes LDS slot i of its 1 KB block, so each lane picks
// the global chunk that belongs in its slot: A slot (r, c) holds chunk
// c ^ ((r >> 1) & 7), B slot (k, c) holds chunk c ^ ((k & 1) << 3), which keeps
// the MFMA fragment reads free of bank conflicts.  Needs K % BK == 0; rows and
// columns past M and N are clamped on load and never stored.
// ---------------------------------------------------------------------------
// Geometry of a global-to-LDS tile: BM x BN outputs, K-steps of one 128-byte
// A row, S LDS stages, WM x WN waves.
template <typename T, int BM, int BN, int WM, int WN, int S>
struct DmaTile {
  static constexpr int NW = WM * WN;
  static constexpr int NT = 64 * NW;
  static constexpr int VE = 16 / sizeof(T);                  // elements per 16-byte chunk
  static constexpr int BK = 128 / sizeof(T);                 // one 128-byte A row per K-step
  static constexpr int TM = BM / WM / 16;
  static constexpr int TN = BN / WN / 16;
  static constexpr int BCH = BN / VE;                        // chunks per B row
  static constexpr int A_LOADS = BM * 8 / NT;                // 16-byte loads per thread per stage
  static constexpr int B_LOADS = BK * BCH / NT;
  static constexpr int STAGE = BM * 128 + BK * BN * static_cast<int>(sizeof(T));   // bytes per stage
  static_assert(TM * WM * 16 == BM && TN * WN * 16 == BN, "tile shape");
  static_assert(A_LOADS * NT == BM * 8 && B_LOADS * NT == BK * BCH, "loads must divide evenly");
  static_assert(BCH % 16 == 0, "B rows must hold a multiple of 16 chunks");
  using Acc = typename Mfma<T>::Acc;
};

// Accumulates K-steps [kt0, kt1) of the tile at (q, m0, n0) into acc (which the
// caller zeroes).  Every wave leaves with its own loads drained; LDS may still
// be read by other waves, so a caller that reuses smem barriers first.
// FB: B is V's standard form, row k0 + k of a K-step at rb[q*K + k0] + k * ldb
// and 16-byte column chunk n at cb[q*N + n] (every K-step inside one affine run
// of rows, every chunk inside one contiguous run of columns).
// AT (with FA): A is K-major in U, element (m, k) at ra[q*M + m] + ca[q*K + k] with
// 16-byte chunks along M; its tile is staged like B's (row k of a K-step at its
// own table entry, one wave-uniform entry per row and load) and read back in the
// MFMA layout from [k][m].
template <typename T, int BM, int BN, int WM, int WN, int S, bool FA, bool FB, bool AT = false>
__device__ __forceinline__ void dma_tile_accumulate(
    const T* __restrict__ A, const T* __restrict__ B, int M, int N, int K, int64_t q, int m0, int n0,
    int kt0, int kt1, const int64_t* __restrict__ ra, const int64_t* __restrict__ ca,
    const int64_t* __restrict__ rb, const int64_t* __restrict__ cb, int64_t ldb, char* smem,
    typename DmaTile<T, BM, BN, WM, WN, S>::Acc (&acc)[DmaTile<T, BM, BN, WM, WN, S>::TM]
                                                      [DmaTile<T, BM, BN, WM, WN, S>::TN]) {
  using D = DmaTile<T, BM, BN, WM, WN, S>;
  constexpr int NT = D::NT, VE = D::VE, BK = D::BK, TM = D::TM, TN = D::TN, BCH = D::BCH;
  constexpr int A_LOADS = D::A_LOADS, B_LOADS = D::B_LOADS, STAGE = D::STAGE;
  const T* Aq = A + (FA ? 0 : q * static_cast<int64_t>(M) * K);
  const T* Bq = B + (FB ? 0 : q * static_cast<int64_t>(K) * N);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  // wave-uniform: LDS destinations of the DMA loads (M0) stay scalar arithmetic
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm0 = (wave / WN) * (BM / WM);
  const int wn0 = (wave % WN) * (BN / WN);

  // Global source of each of this thread's loads (row base, chunk), fixed across K-steps.
  // (K-major A: slot (k, position) of a K-step holds M chunk position ^ ((k & 1) << 3),
  // the lane's M offset fixed, the row offset of k from the step's table entries)
  constexpr int ACH = BM / VE;                    // K-major A: chunks per K row
  static_assert(!AT || (FA && (ACH == 32 || ACH == 64)), "K-major A needs 32 or 64 chunks per row");
  int64_t a_src[A_LOADS];
  int a_chunk[A_LOADS];
#pragma unroll
  for (int i = 0; i < A_LOADS; ++i) {
    const int slot = tid + i * NT;                // A slot = row * 8 + position
    if constexpr (AT) {
      const int k = slot / ACH, c = slot % ACH;
      const int gm = min(m0 + (c ^ ((k & 1) << 3)) * VE, M - VE);
      a_src[i] = ra[q * M + gm];
      a_chunk[i] = 0;
    } else {
      const int r = slot >> 3, c = slot & 7;
      const int gr = min(m0 + r, M - 1);
      a_src[i] = FA ? ra[q * M + gr] : static_cast<int64_t>(gr) * K;
      a_chunk[i] = c ^ ((r >> 1) & 7);
    }
  }
  // K-major A: the row offsets of this thread's K rows of step kt (wave-uniform
  // for 64 chunks per row; two per wave, split by lane half, for 32), one step ahead
  auto at_rows = [&](int kt, int64_t (&rows)[A_LOADS]) {
    const int64_t* tab = ca + q * K + static_cast<int64_t>(kt) * BK;
#pragma unroll
    for (int i = 0; i < A_LOADS; ++i) {
      if constexpr (ACH == 64) {
        rows[i] = tab[wave + i * (NT / 64)];
      } else {
        const int64_t r0 = tab[2 * wave + i * (NT / 32)], r1 = tab[2 * wave + 1 + i * (NT / 32)];
        rows[i] = (lane & 32) ? r1 : r0;
      }
    }
  };
  int64_t arow_next[AT ? A_LOADS : 1];
  if constexpr (AT) {
    if (kt0 < kt1) at_rows(kt0, arow_next);
  }
  int64_t b_src[B_LOADS];
#pragma unroll
  for (int i = 0; i < B_LOADS; ++i) {
    const int slot = tid + i * NT;                // B slot = k * BCH + position
    const int k = slot / BCH, c = slot % BCH;
    const int gch = c ^ ((k & 1) << 3);
    const int gn = min(n0 + gch * VE, N - VE);
    b_src[i] = FB ? static_cast<int64_t>(k) * ldb + cb[q * N + gn] : static_cast<int64_t>(k) * N + gn;
  }
  // Fused A (B): column (row) offset of each K-step, fetched one issue ahead so
  // its latency hides behind the previous step's products.
  int64_t acol_next = FA && !AT && kt0 < kt1 ? ca[q * K + static_cast<int64_t>(kt0) * BK] : 0;
  int64_t brow_next = FB && kt0 < kt1 ? rb[q * K + static_cast<int64_t>(kt0) * BK] : 0;
  auto issue = [&](int kt, int stage) {
    const int k0 = kt * BK;
    int64_t acol = k0;
    int64_t arow[AT ? A_LOADS : 1];
    if constexpr (AT) {
#pragma unroll
      for (int i = 0; i < A_LOADS; ++i) arow[i] = arow_next[i];
      if (kt + 1 < kt1) at_rows(kt + 1, arow_next);
    } else if constexpr (FA) {
      acol = acol_next;
      if (kt + 1 < kt1) acol_next = ca[q * K + static_cast<int64_t>(kt + 1) * BK];
    }
    int64_t brow = static_cast<int64_t>(k0) * N;
    if constexpr (FB) {
      brow = brow_next;
      if (kt + 1 < kt1) brow_next = rb[q * K + static_cast<int64_t>(kt + 1) * BK];
    }
    char* base = smem + stage * STAGE;
#pragma unroll
    for (int i = 0; i < A_LOADS; ++i) {
      if constexpr (AT)
        lds_dma16(Aq + arow[i] + a_src[i], base + (i * NT + wave * 64) * 16);
      else
        lds_dma16(Aq + a_src[i] + acol + a_chunk[i] * VE, base + (i * NT + wave * 64) * 16);
    }
#pragma unroll
    for (int i = 0; i < B_LOADS; ++i)
      lds_dma16(Bq + b_src[i] + brow, base + BM * 128 + (i * NT + wave * 64) * 16);
  };

  const int nk = kt1 - kt0;
#pragma unroll
  for (int s = 0; s < S - 1; ++s)
    if (s < nk) issue(kt0 + s, s);
  for (int it = 0; it < nk; ++it) {
    // step it has landed once at most (S-2) later steps' loads are outstanding
    if (it + S - 2 < nk) wait_vmcnt<(S - 2) * (A_LOADS + B_LOADS)>();
    else wait_vmcnt<0>();
    // a plain barrier: the explicit wait above already covers this wave's loads of
    // step it, and a workgroup fence here would drain the loads still in flight
    asm volatile("s_barrier" ::: "memory");
    if (it + S - 1 < nk) issue(kt0 + it + S - 1, (it + S - 1) % S);
    const char* base = smem + (it % S) * STAGE;
    const T* As = reinterpret_cast<const T*>(base);
    const T* Bs = reinterpret_cast<const T*>(base + BM * 128);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int k = kk + (lane >> 4);
      T a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int m = wm0 + i * 16 + (lane & 15);
        if constexpr (AT)
          a[i] = As[k * BM + ((m / VE) ^ ((k & 1) << 3)) * VE + m % VE];
        else
          a[i] = As[m * BK + ((k / VE) ^ ((m >> 1) & 7)) * VE + k % VE];
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int n = wn0 + j * 16 + (lane & 15);
        b[j] = Bs[k * BN + ((n / VE) ^ ((k & 1) << 3)) * VE + n % VE];
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = Mfma<T>::run(a[i], b[j], acc[i][j]);
    }
  }
}

// Writes a finished tile: C[q] row-major, or scattered through W's offset tables.
template <typename T, int BM, int BN, int WM, int WN, int TM, int TN, bool FC, typename Acc>
__device__ __forceinline__ void store_tile(T* __restrict__ C, int M, int N, int64_t q, int m0, int n0,
                                           const int64_t* __restrict__ rc,
                                           const int64_t* __restrict__ cc, const Acc (&acc)[TM][TN]) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm0 = (wave / WN) * (BM / WM);
  const int wn0 = (wave % WN) * (BN / WN);
  T* Cq = C + (FC ? 0 : q * static_cast<int64_t>(M) * N);
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int col = n0 + wn0 + j * 16 + (lane & 15);
    const int64_t ccol = (FC && col < N) ? cc[q * N + col] : col;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm0 + i * 16 + Mfma<T>::row(lane, r);
        if (row < M && col < N) {
          const int64_t crow = FC ? rc[q * M + row] : static_cast<int64_t>(row) * N;
          Cq[crow + ccol] = acc[i][j][r];
        }
      }
  }
}

// W's offset-table entries of this thread's rows and columns of a tile, loaded
// before the tile's K loop (so their latency hides behind it) and used by
// store_tile_tab.  rows4: W's rows come in contiguous, 16-byte aligned runs of
// a multiple of 4 elements; a binary32 lane then holds 4 consecutive rows of one
// column (rows 4(l/16) .. +3) and writes them with one 16-byte store.
template <int TM, int TN>
struct CTab {
  int64_t row[TM][4];
  int64_t col[TN];
};

template <typename T, int BM, int BN, int WM, int WN, int TM, int TN>
__device__ __forceinline__ void load_ctab(CTab<TM, TN>& t, int M, int N, int64_t q, int m0, int n0,
                                          const int64_t* __restrict__ rc, const int64_t* __restrict__ cc) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm0 = (wave / WN) * (BM / WM);
  const int wn0 = (wave % WN) * (BN / WN);
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int col = n0 + wn0 + j * 16 + (lane & 15);
    t.col[j] = col < N ? cc[q * N + col] : 0;
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = m0 + wm0 + i * 16 + Mfma<T>::row(lane, r);
      t.row[i][r] = row < M ? rc[q * M + row] : 0;
    }
}

template <typename T, int BM, int BN, int WM, int WN, int TM, int TN, typename Acc>
__device__ __forceinline__ void store_tile_tab(T* __restrict__ C, int M, int N, int m0, int n0,
                                               const CTab<TM, TN>& t, bool rows4, const Acc (&acc)[TM][TN]) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm0 = (wave / WN) * (BM / WM);
  const int wn0 = (wave % WN) * (BN / WN);
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int col = n0 + wn0 + j * 16 + (lane & 15);
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      if constexpr (sizeof(T) == 4) {
        const int row0 = m0 + wm0 + i * 16 + Mfma<T>::row(lane, 0);
        if (rows4 && row0 + 3 < M) {
          if (col < N) *reinterpret_cast<f4*>(C + t.row[i][0] + t.col[j]) = acc[i][j];
          continue;
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm0 + i * 16 + Mfma<T>::row(lane, r);
        if (row < M && col < N) C[t.row[i][r] + t.col[j]] = acc[i][j][r];
      }
    }
  }
}

// Piece of a cut tile in accumulator order: element ((wave*TM + i)*TN + j)*4 + r
// of lane l sits at 64 * that + l, so stores and the fixup's loads coalesce.
template <int TM, int TN, typename T, typename Acc>
__device__ __forceinline__ void store_piece(T* __restrict__ piece, const Acc (&acc)[TM][TN]) {
  const int lane = threadIdx.x & 63;
  T* pw = piece + (threadIdx.x >> 6) * (TM * TN * 4 * 64) + lane;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) pw[((i * TN + j) * 4 + r) * 64] = acc[i][j][r];
}

// Stream-K partition: sk_index.hpp.

// Sector product on global-to-LDS tiles.  SK = false: one workgroup per tile
// (XCD-aware order).  SK = true: gridDim.x = 8 * teams_x * ts persistent
// workgroups (teams_x teams of ts on each of the 8 XCDs, which receive
// workgroups round-robin); a tile a team covers whole is written as usual,
// the pieces of a cut tile go to `part` for k_sk_fixup.
// Two-stage 96 x 96 tiles fit three workgroups per CU in LDS; ask the register
// allocator for the matching three waves per SIMD.
template <int BM, int BN, int S>
constexpr int kDmaWavesPerSimd = (S == 2 && BM * BN <= 96 * 96) ? 3 : 1;

template <typename T, int BM, int BN, int WM, int WN, int S, bool FA, bool FB, bool FC, bool SK, bool AT = false>
__global__ __launch_bounds__(64 * WM * WN, (kDmaWavesPerSimd<BM, BN, S>)) void k_gemm_dma(
    const T* __restrict__ A, const T* __restrict__ B, T* __restrict__ C, int M, int N, int K,
    int tiles_m, int tiles_n, int64_t ntiles, const int64_t* __restrict__ ra,
    const int64_t* __restrict__ ca, const int64_t* __restrict__ rc, const int64_t* __restrict__ cc,
    const int64_t* __restrict__ rb, const int64_t* __restrict__ cb, int64_t ldb,
    T* __restrict__ part, int ts, int c_rows4) {
  using D = DmaTile<T, BM, BN, WM, WN, S>;
  constexpr int TM = D::TM, TN = D::TN;
  __shared__ __attribute__((aligned(1024))) char smem[S * D::STAGE];
  typename D::Acc acc[TM][TN];
  const int nk = K / D::BK;
  if constexpr (!SK) {
    const int64_t tile = xcd_remap(blockIdx.x, ntiles);
    int64_t q;
    int tm, tn;
    tile_coords(tile, tiles_m, tiles_n, q, tm, tn);
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = typename D::Acc{};
    // W's table entries ahead of the K loop where registers allow (the binary64
    // 128-wide tiles keep their two waves per SIMD without them)
    constexpr bool kTabAhead = FC && (sizeof(T) == 4 || BM * BN <= 96 * 96);
    CTab<TM, TN> ct;
    if constexpr (kTabAhead) load_ctab<T, BM, BN, WM, WN, TM, TN>(ct, M, N, q, tm * BM, tn * BN, rc, cc);
    dma_tile_accumulate<T, BM, BN, WM, WN, S, FA, FB, AT>(A, B, M, N, K, q, tm * BM, tn * BN, 0, nk, ra, ca,
                                                          rb, cb, ldb, smem, acc);
    if constexpr (kTabAhead)
      store_tile_tab<T, BM, BN, WM, WN, TM, TN>(C, M, N, tm * BM, tn * BN, ct, c_rows4 != 0, acc);
    else
      store_tile<T, BM, BN, WM, WN, TM, TN, FC>(C, M, N, q, tm * BM, tn * BN, rc, cc, acc);
  } else {
    const SkSlot sl = sk_slot(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x), ts);
    const int team = sl.team, member = sl.member, nteam = sl.nteam;
    const int64_t total = ntiles / ts * nk;
    int64_t it = sk_bound(team, total, nteam);
    const int64_t end = sk_bound(team + 1, total, nteam);
    const int64_t first = it / nk;
    while (it < end) {
      const int64_t grp = it / nk;
      const int kt0 = static_cast<int>(it - grp * nk);
      const int kt1 = static_cast<int>(min(static_cast<int64_t>(nk), kt0 + (end - it)));
      const int64_t tile = grp * ts + member;
      const int tn = static_cast<int>(tile % tiles_n);
      const int64_t t2 = tile / tiles_n;
      const int tm = static_cast<int>(t2 % tiles_m);
      const int64_t q = t2 / tiles_m;
      __syncthreads();      // the previous piece's LDS reads are done before new loads land
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = typename D::Acc{};
      dma_tile_accumulate<T, BM, BN, WM, WN, S, FA, FB, AT>(A, B, M, N, K, q, tm * BM, tn * BN, kt0, kt1, ra,
                                                            ca, rb, cb, ldb, smem, acc);
      if (kt0 == 0 && kt1 == nk) {
        if constexpr (FC) {
          // W's table entries all requested before the first store
          CTab<TM, TN> ct;
          load_ctab<T, BM, BN, WM, WN, TM, TN>(ct, M, N, q, tm * BM, tn * BN, rc, cc);
          store_tile_tab<T, BM, BN, WM, WN, TM, TN>(C, M, N, tm * BM, tn * BN, ct, c_rows4 != 0, acc);
        } else {
          store_tile<T, BM, BN, WM, WN, TM, TN, false>(C, M, N, q, tm * BM, tn * BN, rc, cc, acc);
        }
      } else
        store_piece<TM, TN>(part + sk_piece(team, member, ts, grp, first) * (BM * BN), acc);
      it += kt1 - kt0;
    }
  }
}

// Sums the pieces of every tile that stream-K cut, in increasing K order (so
// the result does not depend on scheduling), and writes the tile.  Workgroup
// (tile, chunk) handles the chunk-th of `chunks` equal ranges of the tile's
// elements in accumulator order (a tile spread over many teams -- long K, few
// tiles -- is summed by many workgroups); tiles covered whole by one team
// return at once.  Each element's sum starts from zero and adds the pieces in
// team order: the same arithmetic whatever `chunks` is.
template <typename T, int BM, int BN, int WM, int WN, bool FC>
__global__ __launch_bounds__(64 * WM * WN) void k_sk_fixup(
    const T* __restrict__ part, T* __restrict__ C, int M, int N, int nk, int tiles_m, int tiles_n,
    int64_t ntiles, int ts, int nteam, const int64_t* __restrict__ rc, const int64_t* __restrict__ cc) {
  constexpr int TM = BM / WM / 16, TN = BN / WN / 16;
  constexpr int E = BM * BN;                      // elements of a tile (= of a piece)
  constexpr int PER_WAVE = TM * TN * 4 * 64;
  const int64_t tile = blockIdx.x;
  const int chunks = static_cast<int>(gridDim.y);
  const int64_t grp = tile / ts;
  const int member = static_cast<int>(tile - grp * ts);
  const int64_t total = ntiles / ts * nk;
  const int64_t x0 = grp * nk, x1 = x0 + nk;
  // last team whose share starts at or before x0 (its share is not empty)
  const int64_t t_first = sk_first_team(x0, total, nteam);
  if (sk_bound(t_first + 1, total, nteam) >= x1) return;
  // teams t_first .. t_last hold the tile's pieces (the last one holds iteration
  // x1 - 1); their piece offsets go to LDS once (-1: a team with an empty share)
  constexpr int kList = 1024;
  __shared__ int64_t list[kList];
  const int64_t n_teams = sk_first_team(x1 - 1, total, nteam) - t_first + 1;
  const bool listed = n_teams <= kList;
  if (listed) {
    for (int k = static_cast<int>(threadIdx.x); k < n_teams; k += static_cast<int>(blockDim.x)) {
      const int64_t t = t_first + k;
      const int64_t b0 = sk_bound(t, total, nteam), b1 = sk_bound(t + 1, total, nteam);
      list[k] = b1 > b0 ? sk_piece(static_cast<int>(t), member, ts, grp, b0 / nk) * E : -1;
    }
    __syncthreads();
  }
  const int tn = static_cast<int>(tile % tiles_n);
  const int64_t t2 = tile / tiles_n;
  const int tm = static_cast<int>(t2 % tiles_m);
  const int64_t q = t2 / tiles_m;
  T* Cq = C + (FC ? 0 : q * static_cast<int64_t>(M) * N);
  const int per = (E + chunks - 1) / chunks;
  const int e0 = static_cast<int>(blockIdx.y) * per;
  const int e1 = min(E, e0 + per);
  // accumulator order: element ((w * TM + i) * TN + j) * 4 + r of lane l at 64 * that + l
  // destination of element e of the tile (accumulator order), -1 past M or N;
  // W's table entries are requested before the pieces are read
  auto dest = [&](int e) -> int64_t {
    const int w = e / PER_WAVE;
    const int rem = e - w * PER_WAVE;
    const int lane = rem & 63;
    const int ijr = rem >> 6;
    const int r = ijr & 3;
    const int ij = ijr >> 2;
    const int i = ij / TN, j = ij - (ij / TN) * TN;
    const int row = tm * BM + (w / WN) * (BM / WM) + i * 16 + Mfma<T>::row(lane, r);
    const int col = tn * BN + (w % WN) * (BN / WN) + j * 16 + (lane & 15);
    if (row >= M || col >= N) return -1;
    const int64_t crow = FC ? rc[q * M + row] : static_cast<int64_t>(row) * N;
    const int64_t ccol = FC ? cc[q * N + col] : col;
    return crow + ccol;
  };
  constexpr int NT = 64 * WM * WN;
  constexpr int U = 4;                            // elements in flight per thread
  for (int e = e0 + static_cast<int>(threadIdx.x); e < e1; e += U * NT) {
    T acc[U];
    int64_t dst[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      acc[u] = T(0);
      dst[u] = e + u * NT < e1 ? dest(e + u * NT) : -1;
    }
    if (listed) {
#pragma unroll 4
      for (int k = 0; k < static_cast<int>(n_teams); ++k) {
        const int64_t off = list[k];
        if (off >= 0) {
#pragma unroll
          for (int u = 0; u < U; ++u)
            if (e + u * NT < e1) acc[u] += part[off + e + u * NT];
        }
      }
    } else {
      for (int64_t t = t_first; t < nteam; ++t) {
        const int64_t b0 = sk_bound(t, total, nteam), b1 = sk_bound(t + 1, total, nteam);
        if (b0 >= x1) break;
        if (b1 == b0) continue;
        const int64_t off = sk_piece(static_cast<int>(t), member, ts, grp, b0 / nk) * E;
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (e + u * NT < e1) acc[u] += part[off + e + u * NT];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (dst[u] >= 0) Cq[dst[u]] = acc[u];
  }
}

// ---------------------------------------------------------------------------
// split-bf16: A planes [Q][M][K], B planes [Q][N][K] (K fastest), C f64.
// TA = double or float (fused form): A is read from U's standard reduced form,
// element (q, m, k) at ra[q*M + m] + ca[q*K + k] (every BK-step of K inside one
// contiguous run), VA elements per load, and split into hi/lo in registers the
// way the transforms split it; C goes to W's standard form at
// rc[q*M + m] + cc[q*N + n].
// ---------------------------------------------------------------------------
// FCW: A and B from planes, C to W's standard form through rc / cc.  TC: the
// type C is stored in (binary64 sums rounded to binary32 for a binary32 W, as
// the W transform would round them).
template <int BM, int BN, int BK, int WM, int WN, typename TA = uint16_t, int VA = 8, bool FCW = false,
          typename TC = double>
__global__ __launch_bounds__(64 * WM * WN, (WM * WN == 4 && BK == 32) ? 2 : 1) void k_gemm_bf16x3(
    const uint16_t* __restrict__ Ahi, const uint16_t* __restrict__ Alo,
    const uint16_t* __restrict__ Bhi, const uint16_t* __restrict__ Blo, TC* __restrict__ C,
    int M, int N, int K, int tiles_m, int tiles_n, int64_t ntiles, const TA* __restrict__ U = nullptr,
    const int64_t* __restrict__ ra = nullptr, const int64_t* __restrict__ ca = nullptr,
    const int64_t* __restrict__ rc = nullptr, const int64_t* __restrict__ cc = nullptr) {
  constexpr bool FUSED = !std::is_same<TA, uint16_t>::value;
  constexpr bool FC = FUSED || FCW;
  constexpr int NT = 64 * WM * WN;
  constexpr int V = 8;                // bf16 per 16-byte access
  constexpr int LDK = BK + 8;         // padded row (keeps 16-byte alignment)
  constexpr int TM = BM / WM / 16;
  constexpr int TN = BN / WN / 16;
  static_assert(TM * WM * 16 == BM && TN * WN * 16 == BN, "tile shape");
  static_assert(BK % 32 == 0, "BK");
  static_assert(!FUSED || (VA >= 1 && V % VA == 0 && VA * sizeof(TA) <= 16), "fused A loads");
  constexpr int LA = (BM * BK / V + NT - 1) / NT;
  constexpr int LB = (BN * BK / V + NT - 1) / NT;

  __shared__ uint16_t Ash[2][BM][LDK], Asl[2][BM][LDK];
  __shared__ uint16_t Bsh[2][BN][LDK], Bsl[2][BN][LDK];

  const int64_t tile = xcd_remap(blockIdx.x, ntiles);
  int64_t q;
  int tm, tn;
  tile_coords(tile, tiles_m, tiles_n, q, tm, tn);
  const int64_t offA = q * static_cast<int64_t>(M) * K;
  const int64_t offB = q * static_cast<int64_t>(N) * K;
  static_assert(FC || std::is_same<TC, double>::value, "aligned W is binary64");
  TC* Cq = C + (FC ? 0 : q * static_cast<int64_t>(M) * N);
  const int m0 = tm * BM, n0 = tn * BN;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave / WN) * (BM / WM);
  const int wn0 = (wave % WN) * (BN / WN);

  using V8 = VecT<uint16_t, 8>;
  using VAv = VecT<TA, (FUSED ? VA : 1)>;
  constexpr int NA = FUSED ? V / VA : 1;     // source loads per 8 elements
  V8 rah[LA], ral[LA], rbh[LB], rbl[LB];
  VAv xa[FUSED ? LA : 1][NA];
  // fused A: the standard-form offset of each of this thread's tile rows
  int64_t arow[LA];
#pragma unroll
  for (int i = 0; i < LA; ++i) {
    const int gr = m0 + (tid + i * NT) * V / BK;
    arow[i] = (FUSED && (tid + i * NT) * V < BM * BK && gr < M) ? ra[q * M + gr] : 0;
  }
  auto load_tiles = [&](int k0) {
    const int64_t acol = FUSED ? ca[q * K + k0] : 0;
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int e = (tid + i * NT) * V;
      const int r = e / BK, c = e % BK;
      const int gr = m0 + r, gc = k0 + c;
      if constexpr (FUSED) {
        if (e < BM * BK && gr < M && gc < K) {
#pragma unroll
          for (int j = 0; j < NA; ++j)
            xa[i][j] = *reinterpret_cast<const VAv*>(U + arow[i] + acol + c + j * VA);
        } else {
#pragma unroll
          for (int j = 0; j < NA; ++j)
#pragma unroll
            for (int x = 0; x < VA; ++x) xa[i][j].v[x] = TA(0);
        }
      } else {
        if (e < BM * BK && gr < M && gc < K) {
          const int64_t o = offA + static_cast<int64_t>(gr) * K + gc;
          rah[i] = *reinterpret_cast<const V8*>(Ahi + o);
          ral[i] = *reinterpret_cast<const V8*>(Alo + o);
        } else {
#pragma unroll
          for (int j = 0; j < V; ++j) rah[i].v[j] = ral[i].v[j] = 0;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int e = (tid + i * NT) * V;
      const int r = e / BK, c = e % BK;
      const int gr = n0 + r, gc = k0 + c;
      if (e < BN * BK && gr < N && gc < K) {
        const int64_t o = offB + static_cast<int64_t>(gr) * K + gc;
        rbh[i] = *reinterpret_cast<const V8*>(Bhi + o);
        rbl[i] = *reinterpret_cast<const V8*>(Blo + o);
      } else {
#pragma unroll
        for (int j = 0; j < V; ++j) rbh[i].v[j] = rbl[i].v[j] = 0;
      }
    }
  };
  auto store_tiles = [&](int buf) {
    if constexpr (FUSED) {
#pragma unroll
      for (int i = 0; i < LA; ++i)
#pragma unroll
        for (int j = 0; j < NA; ++j)
#pragma unroll
          for (int x = 0; x < VA; ++x)
            bf16_split(static_cast<double>(xa[i][j].v[x]), rah[i].v[j * VA + x], ral[i].v[j * VA + x]);
    }
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int e = (tid + i * NT) * V;
      if (e < BM * BK) {
        *reinterpret_cast<V8*>(&Ash[buf][e / BK][e % BK]) = rah[i];
        *reinterpret_cast<V8*>(&Asl[buf][e / BK][e % BK]) = ral[i];
      }
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int e = (tid + i * NT) * V;
      if (e < BN * BK) {
        *reinterpret_cast<V8*>(&Bsh[buf][e / BK][e % BK]) = rbh[i];
        *reinterpret_cast<V8*>(&Bsl[buf][e / BK][e % BK]) = rbl[i];
      }
    }
  };

  f4 acc_hh[TM][TN], acc_x[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc_hh[i][j] = acc_x[i][j] = f4{};

  const int nk = (K + BK - 1) / BK;
  load_tiles(0);
  store_tiles(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load_tiles((kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 32) {
      // operand layout of the 16x16x32 bf16 MFMA: lane l holds row (or column)
      // l%16 and the 8 consecutive k values starting at 8*(l/16).
      // A fragments stay in registers for the whole K-step; B fragments are
      // read one column tile at a time to keep register pressure down.
      bf8 ah[TM], al[TM];
      const int kof = kk + 8 * (lane >> 4);
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int r = wm0 + i * 16 + (lane & 15);
        ah[i] = *reinterpret_cast<const bf8*>(&Ash[buf][r][kof]);
        al[i] = *reinterpret_cast<const bf8*>(&Asl[buf][r][kof]);
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int r = wn0 + j * 16 + (lane & 15);
        const bf8 bh = *reinterpret_cast<const bf8*>(&Bsh[buf][r][kof]);
        const bf8 bl = *reinterpret_cast<const bf8*>(&Bsl[buf][r][kof]);
        // the two updates of each cross accumulator are TM products apart
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          acc_hh[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh, acc_hh[i][j], 0, 0, 0);
          acc_x[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl, acc_x[i][j], 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
          acc_x[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh, acc_x[i][j], 0, 0, 0);
      }
    }
    if (kt + 1 < nk) store_tiles(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int col = n0 + wn0 + j * 16 + (lane & 15);
    const int64_t ccol = (FC && col < N) ? cc[q * N + col] : col;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm0 + i * 16 + 4 * (lane >> 4) + r;
        if (row < M && col < N) {
          const int64_t crow = FC ? rc[q * M + row] : static_cast<int64_t>(row) * N;
          Cq[crow + ccol] =
              static_cast<TC>(static_cast<double>(acc_hh[i][j][r]) + static_cast<double>(acc_x[i][j][r]));
        }
      }
  }
}

template <typename T, int BM, int BN, int BK, int WM, int WN>
hipError_t launch_fp(int vec, int64_t batch, int M, int N, int K, const void* A, const void* B,
                     void* C, hipStream_t s, const FusedTables* f, int splits, void* part, size_t part_bytes) {
  const int tiles_m = (M + BM - 1) / BM, tiles_n = (N + BN - 1) / BN;
  const int64_t ntiles = batch * tiles_m * tiles_n;
  const dim3 block(64 * WM * WN);
  const T* a = static_cast<const T*>(A);
  const T* b = static_cast<const T*>(B);
  T* c = static_cast<T*>(C);
  constexpr int VV = 16 / sizeof(T);
  const int64_t* ra = f ? f->ra : nullptr;
  const int64_t* ca = f ? f->ca : nullptr;
  const int64_t* rc = f ? f->rc : nullptr;
  const int64_t* cc = f ? f->cc : nullptr;
  // one vector width for A and B loads: K and N (and for the fused loads, U's runs) must allow it
  const bool fv = vec > 1 && (!f || f->vec > 1);
  // K-major A without M chunks, its contracted modes ending in runs of the vector width
  const bool kv = vec > 1 && f && f->at && !fv && f->a_kvec;
  // split-K only where the workspace holds every partial tile
  if (splits > 1 && (!part || static_cast<size_t>(ntiles) * splits * BM * BN * sizeof(T) > part_bytes)) splits = 1;
  if (splits > 1) {
    T* pt = static_cast<T*>(part);
    const dim3 grid(static_cast<unsigned>(ntiles * splits));
    if (f && f->at && fv)
      hipLaunchKernelGGL((k_gemm<T, BM, BN, BK, WM, WN, VV, true, true, true, true>), grid, block, 0, s, a, b, c,
                         M, N, K, tiles_m, tiles_n, ntiles, ra, ca, rc, cc, pt, splits, f->rb, f->cb, f->ldb,
                         f->krun);
    else if (kv)
      hipLaunchKernelGGL((k_gemm<T, BM, BN, BK, WM, WN, VV, true, true, true, true, true>), grid, block, 0, s, a, b,
                         c, M, N, K, tiles_m, tiles_n, ntiles, ra, ca, rc, cc, pt, splits, f->rb, f->cb, f->ldb,
                         f->krun);
    else if (f && f->at)
      hipLaunchKernelGGL((k_gemm<T, BM, BN, BK, WM, WN, 1, true, true, true, true>), grid, block, 0, s, a, b, c,
                         M, N, K, tiles_m, tiles_n, ntiles, ra, ca, rc, cc, pt, splits, f->rb, f->cb, f->ldb,
                         f->krun);
    else if (f && fv)
      hipLaunchKernelGGL((k_gemm<T, BM, BN, BK, WM, WN, VV, true, true, true>), grid, block, 0, s, a, b, c, M, N,
                         K, tiles_m, tiles_n, ntiles, ra, ca, rc, cc, pt, splits, f->rb, f->cb, f->ldb, f->krun);
    else if (f)
      hipLaunchKernelGGL((k_gemm<T, BM, BN, BK, WM, WN, 1, true, true, true>), grid, block, 0, s, a, b, c, M, N,
                         K, tiles_m, tiles_n, ntiles, ra, ca, rc, cc, pt, splits, f->rb, f->cb, f->ldb, f->krun);
    else if (fv)
      hipLaunchKernelGGL((k_gemm<T, BM, BN, BK, WM, WN, VV, false, false, true>), grid, block, 0, s, a, b, c, M,
                         N, K, tiles_m, tiles_n, ntiles, ra, ca, rc, cc, pt, splits);
    else
      hipLaunchKernelGGL((k_gemm<T, BM, BN, BK, WM, WN, 1, false, false, true>), grid, block, 0, s, a, b, c, M,
                         N, K, tiles_m, tiles_n, ntiles, ra, ca, rc, cc, pt, splits);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // a tile's sum over workgroups of one element per thread (every thread's
    // loads go out together: no second round trip)
    const int64_t max_chunks = std::max<int64_t>(1, static_cast<int64_t>(BM) * BN / (64 * WM * WN));
    const dim3 sgrid(static_cast<unsigned>(ntiles), static_cast<unsigned>(max_chunks));
    if (f)
      hipLaunchKernelGGL((k_split_sum<T, BM, BN, WM, WN, true>), sgrid, block, 0, s, pt, c, M, N, tiles_m,
                         tiles_n, splits, rc, cc);
    else
      hipLaunchKernelGGL((k_split_sum<T, BM, BN, WM, WN, false>), sgrid, block, 0, s, pt, c, M, N, tiles_m,
                         tiles_n, splits, rc, cc);
    return hipGetLastError();
  }
  const dim3 grid(static_cast<unsigned>(ntiles));
  if (f && f->at && fv) {
    hipLaunchKernelGGL((k_gemm<T, BM, BN, BK, WM, WN, VV, true, true, false, true>), grid, block, 0, s, a, b, c,
                       M, N, K, tiles_m, tiles_n, ntiles, ra, ca, rc, cc, nullptr, 1, f->rb, f->cb, f->ldb, f->krun);
  } else if (kv) {
    hipLaunchKernelGGL((k_gemm<T, BM, BN, BK, WM, WN, VV, true, true, false, true, true>), grid, block, 0, s, a, b,
                       c, M, N, K, tiles_m, tiles_n, ntiles, ra, ca, rc, cc, nullptr, 1, f->rb, f->cb, f->ldb,
                       f->krun);
  } else if (f && f->at) {
    hipLaunchKernelGGL((k_gemm<T, BM, BN, BK, WM, WN, 1, true, true, false, true>), grid, block, 0, s, a, b, c,
                       M, N, K, tiles_m, tiles_n, ntiles, ra, ca, rc, cc, nullptr, 1, f->rb, f->cb, f->ldb, f->krun);
  } else if (f && fv) {
    hipLaunchKernelGGL((k_gemm<T, BM, BN, BK, WM, WN, VV, true, true>), grid, block, 0, s, a, b, c,
                       M, N, K, tiles_m, tiles_n, ntiles, ra, ca, rc, cc, nullptr, 1, f->rb, f->cb, f->ldb, f->krun);
  } else if (f) {
    hipLaunchKernelGGL((k_gemm<T, BM, BN, BK, WM, WN, 1, true, true>), grid, block, 0, s, a, b, c,
                       M, N, K, tiles_m, tiles_n, ntiles, ra, ca, rc, cc, nullptr, 1, f->rb, f->cb, f->ldb, f->krun);
  } else if (fv) {
    hipLaunchKernelGGL((k_gemm<T, BM, BN, BK, WM, WN, VV, false, false>), grid, block, 0, s, a, b,
                       c, M, N, K, tiles_m, tiles_n, ntiles, nullptr, nullptr, nullptr, nullptr, nullptr, 1);
  } else {
    hipLaunchKernelGGL((k_gemm<T, BM, BN, BK, WM, WN, 1, false, false>), grid, block, 0, s, a, b, c,
                       M, N, K, tiles_m, tiles_n, ntiles, nullptr, nullptr, nullptr, nullptr, nullptr, 1);
  }
  return hipGetLastError();
}

// Split-bf16 product on global-to-LDS tiles.  A planes (batch, M, K) and B
// planes (batch, N, K) both have K contiguous; a K-step is 32 bf16 = one
// 64-byte row of 4 chunks per operand row and plane, rows XOR-swizzled by
// chunk ((row >> 1) & 3) so that the 16-byte operand reads of 8 consecutive
// rows (one 128-byte bank window) fall on distinct banks; S stages in flight keep the loads S-1 K-steps ahead of the
// products, which a bf16 K-step (48 MFMAs per wave) is too short to hide
// otherwise.  K must be a multiple of 32; rows past M or N are clamped (their
// results are never stored).
// FC: C goes to W's standard form at rc[q*M + m] + cc[q*N + n], stored as TC.
template <int BM, int BN, int WM, int WN, int S, bool FC = false, typename TC = double>
__global__ __launch_bounds__(64 * WM * WN, 1) void k_gemm_bf16x3_dma(
    const uint16_t* __restrict__ Ahi, const uint16_t* __restrict__ Alo,
    const uint16_t* __restrict__ Bhi, const uint16_t* __restrict__ Blo, TC* __restrict__ C,
    int M, int N, int K, int tiles_m, int tiles_n, int64_t ntiles,
    const int64_t* __restrict__ rc = nullptr, const int64_t* __restrict__ cc = nullptr) {
  constexpr int NW = WM * WN;
  constexpr int NT = 64 * NW;
  constexpr int BK = 32;
  constexpr int TM = BM / WM / 16;
  constexpr int TN = BN / WN / 16;
  constexpr int A_LOADS = BM * 8 / NT;            // 16-byte chunks of both A planes per thread
  constexpr int B_LOADS = BN * 8 / NT;
  constexpr int PA = BM * 64, PB = BN * 64;       // bytes per plane per stage
  constexpr int STAGE = 2 * PA + 2 * PB;
  static_assert(TM * WM * 16 == BM && TN * WN * 16 == BN, "tile shape");
  static_assert(A_LOADS * NT == BM * 8 && B_LOADS * NT == BN * 8, "loads must divide evenly");
  __shared__ __attribute__((aligned(1024))) char smem[S * STAGE];

  const int64_t tile = xcd_remap(blockIdx.x, ntiles);
  int64_t q;
  int tm, tn;
  tile_coords(tile, tiles_m, tiles_n, q, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm0 = (wave / WN) * (BM / WM);
  const int wn0 = (wave % WN) * (BN / WN);
  const int64_t offA = q * static_cast<int64_t>(M) * K;
  const int64_t offB = q * static_cast<int64_t>(N) * K;

  // Load slot s = tid + i * NT covers [plane][row][chunk]; the chunk stored at
  // LDS position c of row r comes from global chunk c ^ ((r >> 1) & 3).
  const uint16_t* a_src[A_LOADS];
#pragma unroll
  for (int i = 0; i < A_LOADS; ++i) {
    const int slot = tid + i * NT;
    const int plane = slot / (BM * 4);
    const int rem = slot - plane * (BM * 4);
    const int r = rem >> 2, c = rem & 3;
    const int gr = min(m0 + r, M - 1);
    a_src[i] = (plane ? Alo : Ahi) + offA + static_cast<int64_t>(gr) * K + (c ^ ((r >> 1) & 3)) * 8;
  }
  const uint16_t* b_src[B_LOADS];
#pragma unroll
  for (int i = 0; i < B_LOADS; ++i) {
    const int slot = tid + i * NT;
    const int plane = slot / (BN * 4);
    const int rem = slot - plane * (BN * 4);
    const int r = rem >> 2, c = rem & 3;
    const int gr = min(n0 + r, N - 1);
    b_src[i] = (plane ? Blo : Bhi) + offB + static_cast<int64_t>(gr) * K + (c ^ ((r >> 1) & 3)) * 8;
  }
  auto issue = [&](int kt, int stage) {
    const int k0 = kt * BK;
    char* base = smem + stage * STAGE;
#pragma unroll
    for (int i = 0; i < A_LOADS; ++i) lds_dma16(a_src[i] + k0, base + (i * NT + wave * 64) * 16);
#pragma unroll
    for (int i = 0; i < B_LOADS; ++i) lds_dma16(b_src[i] + k0, base + 2 * PA + (i * NT + wave * 64) * 16);
  };

  f4 acc_hh[TM][TN], acc_x[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc_hh[i][j] = acc_x[i][j] = f4{};

  const int nk = K / BK;
  const int kc = lane >> 4;                       // operand chunk: k = 8 * kc .. 8 * kc + 7
#pragma unroll
  for (int s = 0; s < S - 1; ++s)
    if (s < nk) issue(s, s);
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + S - 2 < nk) wait_vmcnt<(S - 2) * (A_LOADS + B_LOADS)>();
    else wait_vmcnt<0>();
    // a plain barrier: the wait above covers this wave's loads of step kt
    asm volatile("s_barrier" ::: "memory");
    if (kt + S - 1 < nk) issue(kt + S - 1, (kt + S - 1) % S);
    const char* base = smem + (kt % S) * STAGE;
    bf8 ah[TM], al[TM];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const int r = wm0 + i * 16 + (lane & 15);
      const int off = r * 64 + ((kc ^ ((r >> 1) & 3)) << 4);
      ah[i] = *reinterpret_cast<const bf8*>(base + off);
      al[i] = *reinterpret_cast<const bf8*>(base + PA + off);
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int r = wn0 + j * 16 + (lane & 15);
      const int off = 2 * PA + r * 64 + ((kc ^ ((r >> 1) & 3)) << 4);
      const bf8 bh = *reinterpret_cast<const bf8*>(base + off);
      const bf8 bl = *reinterpret_cast<const bf8*>(base + PB + off);
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        acc_hh[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh, acc_hh[i][j], 0, 0, 0);
        acc_x[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl, acc_x[i][j], 0, 0, 0);
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
        acc_x[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh, acc_x[i][j], 0, 0, 0);
    }
  }

  static_assert(FC || std::is_same<TC, double>::value, "aligned W is binary64");
  TC* Cq = C + (FC ? 0 : q * static_cast<int64_t>(M) * N);
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int col = n0 + wn0 + j * 16 + (lane & 15);
    const int64_t ccol = (FC && col < N) ? cc[q * N + col] : col;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm0 + i * 16 + 4 * (lane >> 4) + r;
        if (row < M && col < N) {
          const int64_t crow = FC ? rc[q * M + row] : static_cast<int64_t>(row) * N;
          Cq[crow + ccol] =
              static_cast<TC>(static_cast<double>(acc_hh[i][j][r]) + static_cast<double>(acc_x[i][j][r]));
        }
      }
  }
}

// pa / pb: elements from each hi plane to its lo plane.
// rc / cc: W's offset tables (C written in place), or nullptr (C row-major).
template <int BM, int BN, int WM, int WN, int S>
hipError_t launch_bf16x3_dma(int64_t batch, int M, int N, int K, const void* A, const void* B, void* C,
                             hipStream_t s, int64_t pa, int64_t pb, const int64_t* rc = nullptr,
                             const int64_t* cc = nullptr, int c_bytes = 8) {
  const int tiles_m = (M + BM - 1) / BM, tiles_n = (N + BN - 1) / BN;
  const int64_t ntiles = batch * tiles_m * tiles_n;
  const uint16_t* a = static_cast<const uint16_t*>(A);
  const uint16_t* b = static_cast<const uint16_t*>(B);
  if (rc && c_bytes == 4)
    hipLaunchKernelGGL((k_gemm_bf16x3_dma<BM, BN, WM, WN, S, true, float>), dim3(static_cast<unsigned>(ntiles)),
                       dim3(64 * WM * WN), 0, s, a, a + pa, b, b + pb, static_cast<float*>(C), M, N, K,
                       tiles_m, tiles_n, ntiles, rc, cc);
  else if (rc)
    hipLaunchKernelGGL((k_gemm_bf16x3_dma<BM, BN, WM, WN, S, true>), dim3(static_cast<unsigned>(ntiles)),
                       dim3(64 * WM * WN), 0, s, a, a + pa, b, b + pb, static_cast<double*>(C), M, N, K,
                       tiles_m, tiles_n, ntiles, rc, cc);
  else
    hipLaunchKernelGGL((k_gemm_bf16x3_dma<BM, BN, WM, WN, S>), dim3(static_cast<unsigned>(ntiles)),
                       dim3(64 * WM * WN), 0, s, a, a + pa, b, b + pb, static_cast<double*>(C), M, N, K,
                       tiles_m, tiles_n, ntiles);
  return hipGetLastError();
}

template <int BM, int BN, int BK, int WM, int WN>
hipError_t launch_bf16x3(int64_t batch, int M, int N, int K, const void* A, const void* B, void* C,
                         hipStream_t s, int64_t pa, int64_t pb, const int64_t* rc = nullptr,
                         const int64_t* cc = nullptr, int c_bytes = 8) {
  const int tiles_m = (M + BM - 1) / BM, tiles_n = (N + BN - 1) / BN;
  const int64_t ntiles = batch * tiles_m * tiles_n;
  const dim3 grid(static_cast<unsigned>(ntiles)), block(64 * WM * WN);
  const uint16_t* a = static_cast<const uint16_t*>(A);
  const uint16_t* b = static_cast<const uint16_t*>(B);
  if (rc && c_bytes == 4)
    hipLaunchKernelGGL((k_gemm_bf16x3<BM, BN, BK, WM, WN, uint16_t, 8, true, float>), grid, block, 0, s, a, a + pa,
                       b, b + pb, static_cast<float*>(C), M, N, K, tiles_m, tiles_n, ntiles, nullptr, nullptr,
                       nullptr, rc, cc);
  else if (rc)
    hipLaunchKernelGGL((k_gemm_bf16x3<BM, BN, BK, WM, WN, uint16_t, 8, true>), grid, block, 0, s, a, a + pa, b,
                       b + pb, static_cast<double*>(C), M, N, K, tiles_m, tiles_n, ntiles, nullptr, nullptr,
                       nullptr, rc, cc);
  else
    hipLaunchKernelGGL((k_gemm_bf16x3<BM, BN, BK, WM, WN>), grid, block, 0, s, a, a + pa, b, b + pb,
                       static_cast<double*>(C), M, N, K, tiles_m, tiles_n, ntiles);
  return hipGetLastError();
}

template <int BM, int BN, int BK, int WM, int WN, typename TA, int VA>
void launch_bf16x3_fused_tc(dim3 grid, dim3 block, hipStream_t s, const TA* u, const uint16_t* b, int64_t pb,
                            void* C, int M, int N, int K, int tiles_m, int tiles_n, int64_t ntiles,
                            const FusedTables* f) {
  if (f->c_bytes == 4)
    hipLaunchKernelGGL((k_gemm_bf16x3<BM, BN, BK, WM, WN, TA, VA, false, float>), grid, block, 0, s, nullptr,
                       nullptr, b, b + pb, static_cast<float*>(C), M, N, K, tiles_m, tiles_n, ntiles, u, f->ra,
                       f->ca, f->rc, f->cc);
  else
    hipLaunchKernelGGL((k_gemm_bf16x3<BM, BN, BK, WM, WN, TA, VA>), grid, block, 0, s, nullptr, nullptr, b,
                       b + pb, static_cast<double*>(C), M, N, K, tiles_m, tiles_n, ntiles, u, f->ra, f->ca,
                       f->rc, f->cc);
}

// Fused split-bf16 product: A from U's standard form (binary64 or binary32,
// 16-byte loads where U is 16-byte aligned), C into W's standard form.
template <int BM, int BN, int BK, int WM, int WN>
hipError_t launch_bf16x3_fused(int64_t batch, int M, int N, int K, const void* U, const void* B, void* C,
                               hipStream_t s, int64_t pb, const FusedTables* f) {
  const int tiles_m = (M + BM - 1) / BM, tiles_n = (N + BN - 1) / BN;
  const int64_t ntiles = batch * tiles_m * tiles_n;
  const dim3 grid(static_cast<unsigned>(ntiles)), block(64 * WM * WN);
  const uint16_t* b = static_cast<const uint16_t*>(B);
  if (f->a_bytes == 8) {
    const double* u = static_cast<const double*>(U);
    if (f->vec > 1)
      launch_bf16x3_fused_tc<BM, BN, BK, WM, WN, double, 2>(grid, block, s, u, b, pb, C, M, N, K, tiles_m, tiles_n,
                                                            ntiles, f);
    else
      launch_bf16x3_fused_tc<BM, BN, BK, WM, WN, double, 1>(grid, block, s, u, b, pb, C, M, N, K, tiles_m, tiles_n,
                                                            ntiles, f);
  } else {
    const float* u = static_cast<const float*>(U);
    if (f->vec > 1)
      launch_bf16x3_fused_tc<BM, BN, BK, WM, WN, float, 4>(grid, block, s, u, b, pb, C, M, N, K, tiles_m, tiles_n,
                                                           ntiles, f);
    else
      launch_bf16x3_fused_tc<BM, BN, BK, WM, WN, float, 1>(grid, block, s, u, b, pb, C, M, N, K, tiles_m, tiles_n,
                                                           ntiles, f);
  }
  return hipGetLastError();
}

// Compute units of the current device (cached per device).
int device_cus() {
  static std::atomic<int> cus[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int n = cus[dev].load(std::memory_order_relaxed);
  if (n == 0) {
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) n = 256;
    cus[dev].store(n, std::memory_order_relaxed);
  }
  return n;
}

// Fused mode of a global-to-LDS product: 0 aligned operands, 1 A read from U and
// C written to W in place, 2 B read from V in place as well; 3 and 4: as 1 and 2
// with A K-major in U (128-row tiles only).
inline int dma_mode(const FusedTables* f) { return !f ? 0 : (f->rb ? 2 : 1) + (f->at ? 2 : 0); }

template <typename T, int BM, int BN, int WM, int WN, int S, bool SK>
hipError_t launch_dma_kernel(int mode, dim3 grid, dim3 block, hipStream_t s, const T* a, const T* b, T* c,
                             int M, int N, int K, int tiles_m, int tiles_n, int64_t ntiles,
                             const FusedTables* f, T* pt, int ts) {
  const int64_t* ra = f ? f->ra : nullptr;
  const int64_t* ca = f ? f->ca : nullptr;
  const int64_t* rc = f ? f->rc : nullptr;
  const int64_t* cc = f ? f->cc : nullptr;
  const int64_t* rb = f ? f->rb : nullptr;
  const int64_t* cb = f ? f->cb : nullptr;
  const int64_t ldb = f ? f->ldb : 0;
  const int rows4 = f && f->c_rows4 && (reinterpret_cast<uintptr_t>(c) & 15) == 0 ? 1 : 0;
  if constexpr (BM == 128) {
    if (mode == 4) {
      hipLaunchKernelGGL((k_gemm_dma<T, BM, BN, WM, WN, S, true, true, true, SK, true>), grid, block, 0, s, a, b, c,
                         M, N, K, tiles_m, tiles_n, ntiles, ra, ca, rc, cc, rb, cb, ldb, pt, ts, rows4);
      return hipGetLastError();
    }
    if (mode == 3) {
      hipLaunchKernelGGL((k_gemm_dma<T, BM, BN, WM, WN, S, true, false, true, SK, true>), grid, block, 0, s, a, b,
                         c, M, N, K, tiles_m, tiles_n, ntiles, ra, ca, rc, cc, rb, cb, ldb, pt, ts, rows4);
      return hipGetLastError();
    }
  } else {
    if (mode > 2) return hipErrorInvalidValue;   // K-major A takes 128-row tiles only
  }
  if (mode == 2)
    hipLaunchKernelGGL((k_gemm_dma<T, BM, BN, WM, WN, S, true, true, true, SK>), grid, block, 0, s, a, b, c, M,
                       N, K, tiles_m, tiles_n, ntiles, ra, ca, rc, cc, rb, cb, ldb, pt, ts, rows4);
  else if (mode == 1)
    hipLaunchKernelGGL((k_gemm_dma<T, BM, BN, WM, WN, S, true, false, true, SK>), grid, block, 0, s, a, b, c, M,
                       N, K, tiles_m, tiles_n, ntiles, ra, ca, rc, cc, rb, cb, ldb, pt, ts, rows4);
  else
    hipLaunchKernelGGL((k_gemm_dma<T, BM, BN, WM, WN, S, false, false, false, SK>), grid, block, 0, s, a, b, c,
                       M, N, K, tiles_m, tiles_n, ntiles, ra, ca, rc, cc, rb, cb, ldb, pt, ts, rows4);
  return hipGetLastError();
}

// part / part_bytes: stream-K piece buffer (nullptr: one workgroup per tile).
template <typename T, int BM, int BN, int WM, int WN, int S>
hipError_t launch_dma(int64_t batch, int M, int N, int K, const void* A, const void* B, void* C,
                      hipStream_t s, const FusedTables* f, void* part, size_t part_bytes) {
  // B rows must hold a multiple of 16 chunks of 16 bytes (the swizzle works in
  // halves of a bank cycle); other shapes are never selected for this type.
  if constexpr ((BN * sizeof(T) / 16) % 16 != 0) {
    return hipErrorInvalidValue;
  } else {
  const int tiles_m = (M + BM - 1) / BM, tiles_n = (N + BN - 1) / BN;
  const int64_t ntiles = batch * tiles_m * tiles_n;
  const dim3 block(64 * WM * WN);
  const T* a = static_cast<const T*>(A);
  const T* b = static_cast<const T*>(B);
  T* c = static_cast<T*>(C);
  const int64_t* rc = f ? f->rc : nullptr;
  const int64_t* cc = f ? f->cc : nullptr;
  const int mode = dma_mode(f);
  const int nk = K / DmaTile<T, BM, BN, WM, WN, S>::BK;
  int P = 0, ts = 1;
  if (part) {
    // resident workgroups per CU of this instantiation (per fused mode), cached
    static std::atomic<int> occupancy[5];
    int occ = occupancy[mode].load(std::memory_order_relaxed);
    if (occ == 0) {
      // (the K-major forms have the same LDS and about the same registers)
      auto kern = mode % 2 == 0 && mode > 0 ? k_gemm_dma<T, BM, BN, WM, WN, S, true, true, true, true>
                  : mode > 0              ? k_gemm_dma<T, BM, BN, WM, WN, S, true, false, true, true>
                                          : k_gemm_dma<T, BM, BN, WM, WN, S, false, false, false, true>;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 64 * WM * WN, 0) != hipSuccess || occ < 1)
        occ = 1;
      occupancy[mode].store(occ, std::memory_order_relaxed);
    }
    // no more persistent workgroups than resident ones, nor than the pieces buffer holds
    const SkLaunch sl = sk_launch(ntiles, tiles_n, nk,
                                  std::min<int64_t>(kSkSlots, static_cast<int64_t>(device_cus()) * occ),
                                  static_cast<int64_t>(part_bytes / sizeof(T)), static_cast<int64_t>(BM) * BN,
                                  kSkMinIters);
    P = sl.P;
    ts = sl.ts;
  }
  T* pt = static_cast<T*>(part);
  if (P > 0) {
    const int nteam = P / ts;
    hipError_t e = launch_dma_kernel<T, BM, BN, WM, WN, S, true>(mode, dim3(P), block, s, a, b, c, M, N, K,
                                                                 tiles_m, tiles_n, ntiles, f, pt, ts);
    if (e != hipSuccess) return e;
    // a tile spans about nk / (iterations per team) + 1 teams' pieces: the sum of
    // a tile goes to enough workgroups that each thread makes one pass of four
    // elements (their loads in flight together), more when the tile has many
    // pieces, down to one element per thread
    const int64_t per_team = std::max<int64_t>(1, (ntiles / ts) * nk / nteam);
    const int64_t spans = nk / per_team + 1;
    const int64_t max_chunks = std::max<int64_t>(1, static_cast<int64_t>(BM) * BN / (64 * WM * WN));
    const int64_t one_pass = std::max<int64_t>(1, max_chunks / 4);
    const dim3 fgrid(static_cast<unsigned>(ntiles),
                     static_cast<unsigned>(std::min<int64_t>(max_chunks, std::max<int64_t>(one_pass, spans))));
    if (f)
      hipLaunchKernelGGL((k_sk_fixup<T, BM, BN, WM, WN, true>), fgrid, block, 0, s, pt, c, M, N, nk, tiles_m,
                         tiles_n, ntiles, ts, nteam, rc, cc);
    else
      hipLaunchKernelGGL((k_sk_fixup<T, BM, BN, WM, WN, false>), fgrid, block, 0, s, pt, c, M, N, nk, tiles_m,
                         tiles_n, ntiles, ts, nteam, rc, cc);
    return hipGetLastError();
  }
  return launch_dma_kernel<T, BM, BN, WM, WN, S, false>(mode, dim3(static_cast<unsigned>(ntiles)), block, s, a,
                                                        b, c, M, N, K, tiles_m, tiles_n, ntiles, f, pt, 1);
  }
}

// One f64/f32 tile configuration.  dma: direct global->LDS loads into an
// S-stage ring (needs K to be a multiple of the 128-byte K-depth and N a
// multiple of 16 bytes).
// Dispatch order = the tile table of choose_fp_gemm.
template <typename T>
hipError_t launch_fp_tile(int idx, int vec, int64_t batch, int M, int N, int K, const void* A,
                          const void* B, void* C, hipStream_t s, const FusedTables* f, void* part,
                          size_t part_bytes, int splits) {
  switch (idx) {
    case 0: return launch_fp<T, 128, 128, 16, 2, 2>(vec, batch, M, N, K, A, B, C, s, f, splits, part, part_bytes);
    case 1: return launch_fp<T, 128, 96, 16, 2, 2>(vec, batch, M, N, K, A, B, C, s, f, splits, part, part_bytes);
    case 2: return launch_fp<T, 128, 64, 16, 2, 2>(vec, batch, M, N, K, A, B, C, s, f, splits, part, part_bytes);
    case 3: return launch_fp<T, 128, 48, 16, 4, 1>(vec, batch, M, N, K, A, B, C, s, f, splits, part, part_bytes);
    case 4: return launch_fp<T, 96, 96, 16, 2, 2>(vec, batch, M, N, K, A, B, C, s, f, splits, part, part_bytes);
    case 5: return launch_fp<T, 64, 96, 16, 2, 2>(vec, batch, M, N, K, A, B, C, s, f, splits, part, part_bytes);
    case 6: return launch_dma<T, 128, 128, 2, 2, 2>(batch, M, N, K, A, B, C, s, f, part, part_bytes);
    case 7: return launch_dma<T, 128, 96, 2, 2, 2>(batch, M, N, K, A, B, C, s, f, part, part_bytes);
    case 8: return launch_dma<T, 128, 64, 2, 2, 3>(batch, M, N, K, A, B, C, s, f, part, part_bytes);
    case 9: return launch_dma<T, 96, 96, 2, 2, 3>(batch, M, N, K, A, B, C, s, f, part, part_bytes);
    default: return launch_dma<T, 96, 96, 2, 2, 2>(batch, M, N, K, A, B, C, s, f, part, part_bytes);
  }
}

}  // namespace

// Row-streaming product for K and N at most 64 (gemm_rows.hip).
hipError_t launch_gemm_rows(bool f64, int64_t batch, int M, int N, int K, const void* A, const void* B, void* C,
                            hipStream_t s, const FusedTables* f);
// Long-K product for M and N at most 64 (gemm_tallk.hip).
hipError_t launch_gemm_tallk(bool f64, int64_t batch, int M, int N, int K, const void* A, const void* B, void* C,
                             hipStream_t s, const FusedTables* f, void* part, int ranges);

// Wide split-bf16 tiles with one binary32 accumulator (gemm_bf16x3.hip).
hipError_t launch_bf16x3_wide(int variant, int64_t batch, int M, int N, int K, const void* A, const void* B,
                              void* C, hipStream_t s, int64_t pa, int64_t pb, const int64_t* rc,
                              const int64_t* cc, int c_bytes, bool il, const int64_t* ra, const int64_t* ca);

// plane_a / plane_b (split-bf16 only): elements from a hi plane to its lo
// plane, 0 for the packed layout (batch * m * k, batch * n * k).  il
// (split-bf16 only): both operands' planes interleaved by 32-deep K-steps, which
// only the wide tiles read.
int launch_sector_gemm(int compute, int64_t batch, int64_t m, int64_t k, int64_t n, const void* A,
                       const void* B, void* C, hipStream_t stream, std::string* err,
                       const FusedTables* fused, void* part, size_t part_bytes, int64_t plane_a,
                       int64_t plane_b, bool il) {
  if (batch == 0 || m == 0 || n == 0) return SYMT_OK;
  if (m > INT32_MAX || n > INT32_MAX || k > INT32_MAX) {
    if (err) *err = "sector product dimension above 2^31-1";
    return SYMT_EUNSUPPORTED;
  }
  const int M = static_cast<int>(m), N = static_cast<int>(n), K = static_cast<int>(k);
  hipError_t e = hipSuccess;
  if (compute == SYMT_COMPUTE_BF16X3) {
    if (K % 8 != 0) {
      if (err) *err = "split-bf16 product needs the contracted extent to be a multiple of 8";
      return SYMT_EUNSUPPORTED;
    }
    const char* forced = std::getenv("SYMT_GEMM_TILE");
    const std::string f = forced ? forced : "";
    const bool dma_ok = K % 32 == 0;
    const int64_t pa = plane_a > 0 ? plane_a : batch * static_cast<int64_t>(M) * K;
    const int64_t pb = plane_b > 0 ? plane_b : batch * static_cast<int64_t>(N) * K;
    const int64_t* wrc = fused ? fused->rc : nullptr;   // C in place (planes for A and B)
    const int64_t* wcc = fused ? fused->cc : nullptr;
    const int wcb = fused ? fused->c_bytes : 8;           // W's element size
    if (il) {
      // the planner interleaves the planes only where a wide tile runs; with U's
      // tables (fused->ra) the 256 x 256 tile reads A as binary32 U in place
      const int wv = f == "bw256x128s3" ? 1 : f == "bw256x256s2" ? 0 : f.empty() ? bf16x3_wide_tile(batch, M, N) : -1;
      const bool fa = fused && fused->ra;
      if (!dma_ok || wv < 0 || (fa && (wv != 0 || fused->a_bytes != 4 || !fused->ca || !wrc))) {
        if (err) *err = "interleaved split-bf16 planes need a wide tile and whole 32-deep K-steps";
        return SYMT_EUNSUPPORTED;
      }
      e = launch_bf16x3_wide(wv, batch, M, N, K, A, B, C, stream, pa, pb, wrc, wcc, wcb, true,
                             fa ? fused->ra : nullptr, fa ? fused->ca : nullptr);
    } else if (fused && fused->ra) {
      // register tiles only (the planner fuses where the launcher would pick one)
      if (!bf16x3_register_tile(M, N, K) || K % 32 != 0) {
        if (err) *err = "fused split-bf16 product needs a register tile and whole 32-deep K-steps";
        return SYMT_EUNSUPPORTED;
      }
      const int t = bf16x3_fused_tile(M, N);
      e = t == 0   ? launch_bf16x3_fused<128, 64, 32, 4, 1>(batch, M, N, K, A, B, C, stream, pb, fused)
          : t == 2 ? launch_bf16x3_fused<128, 256, 32, 2, 4>(batch, M, N, K, A, B, C, stream, pb, fused)
          : t == 3 ? launch_bf16x3_fused<128, 96, 32, 2, 2>(batch, M, N, K, A, B, C, stream, pb, fused)
                   : launch_bf16x3_fused<128, 128, 32, 2, 2>(batch, M, N, K, A, B, C, stream, pb, fused);
    } else if (f == "bw256x256s2" && dma_ok) e = launch_bf16x3_wide(0, batch, M, N, K, A, B, C, stream, pa, pb, wrc, wcc, wcb, false, nullptr, nullptr);
    else if (f == "bw256x128s3" && dma_ok) e = launch_bf16x3_wide(1, batch, M, N, K, A, B, C, stream, pa, pb, wrc, wcc, wcb, false, nullptr, nullptr);
    else if (f == "bd256x128s3" && dma_ok) e = launch_bf16x3_dma<256, 128, 4, 2, 3>(batch, M, N, K, A, B, C, stream, pa, pb, wrc, wcc, wcb);
    else if (f == "bd128x256s3" && dma_ok) e = launch_bf16x3_dma<128, 256, 2, 4, 3>(batch, M, N, K, A, B, C, stream, pa, pb, wrc, wcc, wcb);
    else if (f == "b128x128k64") e = launch_bf16x3<128, 128, 64, 2, 2>(batch, M, N, K, A, B, C, stream, pa, pb, wrc, wcc, wcb);
    else if (f == "b128x128k32") e = launch_bf16x3<128, 128, 32, 2, 2>(batch, M, N, K, A, B, C, stream, pa, pb, wrc, wcc, wcb);
    else if (f == "b256x128k32") e = launch_bf16x3<256, 128, 32, 4, 2>(batch, M, N, K, A, B, C, stream, pa, pb, wrc, wcc, wcb);
    else if (f == "b128x256k32") e = launch_bf16x3<128, 256, 32, 2, 4>(batch, M, N, K, A, B, C, stream, pa, pb, wrc, wcc, wcb);
    else if (f == "b128x64k32") e = launch_bf16x3<128, 64, 32, 4, 1>(batch, M, N, K, A, B, C, stream, pa, pb, wrc, wcc, wcb);
    else if (f == "b128x96k32") e = launch_bf16x3<128, 96, 32, 2, 2>(batch, M, N, K, A, B, C, stream, pa, pb, wrc, wcc, wcb);
    else if (f == "b64x64k32") e = launch_bf16x3<64, 64, 32, 2, 2>(batch, M, N, K, A, B, C, stream, pa, pb, wrc, wcc, wcb);
    else if (dma_ok && f.empty() && bf16x3_wide_tile(batch, M, N) >= 0)
      e = launch_bf16x3_wide(bf16x3_wide_tile(batch, M, N), batch, M, N, K, A, B, C, stream, pa, pb, wrc, wcc, wcb, false,
                             nullptr, nullptr);
    else if (dma_ok && f.empty() && M >= 256 && N >= 512)
      e = launch_bf16x3_dma<128, 256, 2, 4, 3>(batch, M, N, K, A, B, C, stream, pa, pb, wrc, wcc, wcb);
    else if (N <= 64)
      e = launch_bf16x3<128, 64, 32, 4, 1>(batch, M, N, K, A, B, C, stream, pa, pb, wrc, wcc, wcb);
    else if (N >= 1024 && M >= 1024)
      e = launch_bf16x3<128, 256, 32, 2, 4>(batch, M, N, K, A, B, C, stream, pa, pb, wrc, wcc, wcb);
    else if ((N + 95) / 96 * 96 - N < (N + 127) / 128 * 128 - N)   // fewer padded columns
      e = launch_bf16x3<128, 96, 32, 2, 2>(batch, M, N, K, A, B, C, stream, pa, pb, wrc, wcc, wcb);
    else
      e = launch_bf16x3<128, 128, 32, 2, 2>(batch, M, N, K, A, B, C, stream, pa, pb, wrc, wcc, wcb);
  } else {
    const bool f64 = compute == SYMT_COMPUTE_F64;
    const int vw = f64 ? 2 : 4;
    const int vec = (K % vw == 0 && N % vw == 0) ? vw : 1;
    // K stepped run by run (fused->krun) needs the register tiles; K-major A
    // (fused->at) with 16-byte chunks takes the 128-row global-to-LDS tiles too
    const bool a_kmajor = fused && fused->at;
    const bool aligned = (reinterpret_cast<uintptr_t>(A) & 15) == 0 &&
                         (reinterpret_cast<uintptr_t>(B) & 15) == 0 &&
                         (!fused || (fused->vec > 1 && fused->krun == 0));
    const GemmChoice gc = choose_fp_gemm(batch, M, N, K, f64 ? 8 : 4, aligned, a_kmajor);
    if (gc.tile == kTallKTile) {
      // without room for the partials (the allocation-free entry point may drop
      // them) the 128 x 48 register tile runs instead, one workgroup per tile
      const bool room = part && part_bytes >= gc.partial_bytes;
      e = room ? launch_gemm_tallk(f64, batch, M, N, K, A, B, C, stream, fused, part, gc.splits)
          : f64 ? launch_fp_tile<double>(3, vec, batch, M, N, K, A, B, C, stream, fused, nullptr, 0, 1)
                : launch_fp_tile<float>(3, vec, batch, M, N, K, A, B, C, stream, fused, nullptr, 0, 1);
      if (e != hipSuccess) {
        if (err) *err = std::string("sector product launch: ") + hipGetErrorString(e);
        return SYMT_EHIP;
      }
      return SYMT_OK;
    }
    if ((!gc.sk && gc.splits <= 1) || (reinterpret_cast<uintptr_t>(part) & 15) != 0) part = nullptr;
    e = gc.tile == kRowsTile ? launch_gemm_rows(f64, batch, M, N, K, A, B, C, stream, fused)
        : f64 ? launch_fp_tile<double>(gc.tile, vec, batch, M, N, K, A, B, C, stream, fused, part, part_bytes,
                                     gc.splits)
            : launch_fp_tile<float>(gc.tile, vec, batch, M, N, K, A, B, C, stream, fused, part, part_bytes,
                                    gc.splits);
  }
  if (e != hipSuccess) {
    if (err) *err = std::string("sector product launch: ") + hipGetErrorString(e);
    return SYMT_EHIP;
  }
  return SYMT_OK;
}

}  // namespace symt

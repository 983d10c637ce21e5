// Row-streaming sector product for short contractions (Alg. 2's product step
// where K and N are both at most 64): C[Q] = A[Q] B[Q] with A[Q] tall (M rows),
// f64 or f32.
//
// Such a product moves 8 (K + N) bytes per row of A and C for 2 K N flops, so
// it is bound by HBM (about 6 flops per byte at K = N = 48), not by the matrix
// cores.  This kernel therefore reads every element of A exactly once, straight
// from global memory into the MFMA operand registers (no LDS staging of A),
// keeps all of B[Q] in LDS for the workgroup's lifetime, and writes C straight
// from the accumulators.  Each wave owns blocks of 16 (binary64) or 32 (binary32) rows by all N columns and
// issues the loads of a whole block (K / 4 per 16-row group) before its first
// MFMA, and the next block's loads before this block's MFMAs (table reads run
// further ahead); waves run their row blocks independently (one barrier, after
// B is in LDS).
//
// Operands are addressed through separable offset tables, so the same kernel
// reads A from U's standard form (row offsets ra, column offsets ca, any
// layout of U's modes), B from V's (rb, cb) and writes C into W's (rc, cc);
// a null table stands for the aligned row-major form.  K is summed four
// indices per MFMA (v_mfma_f64_16x16x4_f64, v_mfma_f32_16x16x4_f32): in order in
// binary64, in a fixed order within groups of 16 in binary32 (see below).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "gemm_common.hpp"
#include "plan.hpp"

namespace symt {

namespace {

template <typename T>
struct RowMfma;
// Accumulator rows (lane l, item r; column l % 16): f64 l/16 + 4r, f32 4(l/16) + r.
template <>
struct RowMfma<double> {
  using Acc = d4;
  static __device__ __forceinline__ Acc run(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct RowMfma<float> {
  using Acc = f4;
  static __device__ __forceinline__ Acc run(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

constexpr int kRowWaves = 4;     // waves per workgroup

// 16-row groups per wave block: one for binary64 (its A, accumulators and
// prefetched A fill two thirds of the registers already), two for binary32
// (each B value read from LDS then feeds two MFMAs)
template <typename T, int KS, int TN>
constexpr int row_groups() {
  return sizeof(T) == 8 ? 1 : 2;
}

// KS: K-steps of 4 (K <= 4 KS); TN: 16-column tiles (N <= 16 TN).
// Grid: (workgroups per Q, Q).  Wave w of workgroup x walks row blocks
// x * kRowWaves + w, stepping by gridDim.x * kRowWaves.
// TR: the MFMA computes the transposed tile (B^T A^T), so that each lane's
// accumulators hold one row of C and a store instruction writes 16 consecutive
// rows (for a W whose rows, not columns, are its contiguous index).
// RV > 1 (A's rows contiguous in aligned runs of RV, as where U's output modes
// trail: A read K-major): lane r of a 16 x RV-row group loads rows RV r ..
// RV r + RV - 1 of one K index with one 16-byte load and feeds them to RV
// MFMAs, whose output row p then stands for row RV p + t of the group.
// Binary32 steps through K in groups of 16: K-step 4 u + t takes index
// 16 u + 4 kq + t at lane group kq (the same sums as 4 s + kq, permuted within
// each group, in every variant); KV = 4 (A's K index contiguous in aligned
// runs of 4): lane (r, kq) loads the four indices 16 u + 4 kq .. + 3 of its row
// with one 16-byte load for K-steps 4 u .. 4 u + 3.
template <typename T, int KS, int TN, bool TR, int RV = 1, int KV = 1>
__global__ __launch_bounds__(64 * kRowWaves, (RV > 1 ? 2 : 1)) void k_gemm_rows(
    const T* __restrict__ A, const T* __restrict__ B, T* __restrict__ C, int M, int N, int K,
    const int64_t* __restrict__ ra, const int64_t* __restrict__ ca, const int64_t* __restrict__ rb,
    const int64_t* __restrict__ cb, const int64_t* __restrict__ rc, const int64_t* __restrict__ cc) {
  using Acc = typename RowMfma<T>::Acc;
  static_assert(RV == 1 || (!TR && RV * sizeof(T) == 16), "row vectors: 16 bytes, lanes along columns");
  constexpr int kRowGroups = RV > 1 ? 1 : row_groups<T, KS, TN>();
  constexpr int NG = kRowGroups * RV;            // 16-row MFMA groups per block
  constexpr int KP = 4 * KS;
  constexpr int NP = 16 * TN;
  // B rows padded so that the four k-rows of one operand read start 16 * sizeof(T)
  // bytes apart modulo the 256-byte bank cycle
  constexpr int ROWB = NP * static_cast<int>(sizeof(T));
  constexpr int SHIFT = 16 * static_cast<int>(sizeof(T));
  constexpr int PADB = ((SHIFT - ROWB % 256 + 256) % 256) / static_cast<int>(sizeof(T));
  __shared__ T Bs[KP][NP + PADB];
  __shared__ int64_t cols_a[KP];

  const int64_t q = blockIdx.y;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

  // B[Q] (zero past K and N) and A's column offsets (past K: never read)
  for (int e = tid; e < KP * NP; e += 64 * kRowWaves) {
    const int k = e / NP, n = e - (e / NP) * NP;
    T x = T(0);
    if (k < K && n < N)
      x = rb ? B[rb[q * K + k] + cb[q * N + n]] : B[(q * K + k) * static_cast<int64_t>(N) + n];
    Bs[k][n] = x;
  }
  for (int k = tid; k < KP; k += 64 * kRowWaves)
    cols_a[k] = k < K ? (ca ? ca[q * K + k] : static_cast<int64_t>(k)) : 0;
  __syncthreads();

  // this lane's output columns: one per 16-column tile, or (TR) four per tile
  constexpr int NC = TR ? 4 : 1;
  int64_t ccol[TN][NC];
#pragma unroll
  for (int j = 0; j < TN; ++j)
#pragma unroll
    for (int r = 0; r < NC; ++r) {
      const int col = j * 16 + (TR ? RowMfma<T>::row(lane, r) : (lane & 15));
      ccol[j][r] = col < N ? (cc ? cc[q * N + col] : static_cast<int64_t>(col)) : -1;
    }
  const int kq = lane >> 4;                      // k index within each K-step
  const int64_t blocks = (M + 16 * NG - 1) / (16 * NG);
  const int64_t step = static_cast<int64_t>(gridDim.x) * kRowWaves;
  // Row offsets of block b's A rows (this lane's row of each 16-row group) and
  // of its C rows (this lane's accumulator rows; -1 past M).
  auto a_rows = [&](int64_t b, int64_t (&rbase)[kRowGroups]) {
#pragma unroll
    for (int i = 0; i < kRowGroups; ++i) {
      const int m = min(static_cast<int>(b * 16 * NG) + i * 16 * RV + RV * (lane & 15), M - RV);
      rbase[i] = ra ? ra[q * M + m] : (q * M + m) * static_cast<int64_t>(K);
    }
  };
  constexpr int NR = TR ? 1 : 4;                 // C rows per lane and row group
  auto c_rows = [&](int64_t b, int64_t (&crow)[NG][NR]) {
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int i = g / RV, t = g % RV;
        const int row = static_cast<int>(b * 16 * NG) + i * 16 * RV +
                        (TR ? (lane & 15) : RV * RowMfma<T>::row(lane, r) + t);
        crow[g][r] = row < M ? (rc ? rc[q * M + row] : (q * M + row) * static_cast<int64_t>(N)) : -1;
      }
  };
  // A: lane (r, kq) of group i holds A[m0 + 16 RV i + RV r + t][4 s + kq], t < RV, for every step s
  static_assert(KV == 1 || (RV == 1 && KV * sizeof(T) == 16 && KS % KV == 0), "K vectors: 16 bytes");
  // K index of (step s, lane group kq): binary64 4 s + kq; binary32 16 (s / 4) + 4 kq + s % 4
  constexpr int KO = sizeof(T) == 4 ? 4 : 1;
  static_assert(KS % KO == 0, "whole groups of K-steps");
  auto kidx = [&](int s) { return KO > 1 ? 4 * KO * (s / KO) + KO * kq + s % KO : 4 * s + kq; };
  using AV = VecT<T, RV>;
  auto load_a = [&](const int64_t (&rbase)[kRowGroups], AV (&a)[kRowGroups][KS]) {
#pragma unroll
    for (int i = 0; i < kRowGroups; ++i) {
      if constexpr (KV > 1) {
#pragma unroll
        for (int u = 0; u < KS / KV; ++u) {
          const int k = kidx(KV * u);
          VecT<T, KV> x;
          if (k < K) {
            x = *reinterpret_cast<const VecT<T, KV>*>(A + rbase[i] + cols_a[k]);
          } else {
#pragma unroll
            for (int t = 0; t < KV; ++t) x.v[t] = T(0);
          }
#pragma unroll
          for (int t = 0; t < KV; ++t) a[i][KV * u + t].v[0] = x.v[t];
        }
      } else {
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const int k = kidx(s);
          if (k < K) {
            a[i][s] = *reinterpret_cast<const AV*>(A + rbase[i] + cols_a[k]);
          } else {
#pragma unroll
            for (int t = 0; t < RV; ++t) a[i][s].v[t] = T(0);
          }
        }
      }
    }
  };
  int64_t blk = static_cast<int64_t>(blockIdx.x) * kRowWaves + wave;
  if (blk >= blocks) return;
  // Loads run ahead: A one block ahead, its row offsets two blocks ahead, and
  // each block's C row offsets before its products, so no table read waits on
  // the critical path (the loads complete in issue order).
  AV a[kRowGroups][KS], an[kRowGroups][KS];
  int64_t r1[kRowGroups], r2[kRowGroups];
  a_rows(blk, r1);
  load_a(r1, a);
  if (blk + step < blocks) a_rows(blk + step, r1);
  for (; blk < blocks; blk += step) {
    int64_t crow[NG][NR];
    c_rows(blk, crow);
    const bool more = blk + step < blocks;
    if (blk + 2 * step < blocks) a_rows(blk + 2 * step, r2);
    if (more) load_a(r1, an);
    Acc acc[NG][TN];
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[g][j] = Acc{};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const T b = Bs[kidx(s)][j * 16 + (lane & 15)];
#pragma unroll
        for (int g = 0; g < NG; ++g) {
          const T av = a[g / RV][s].v[g % RV];
          acc[g][j] = TR ? RowMfma<T>::run(b, av, acc[g][j]) : RowMfma<T>::run(av, b, acc[g][j]);
        }
      }
    }
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t cr = crow[g][TR ? 0 : r];
        if (cr < 0) continue;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int64_t cc_ = ccol[j][TR ? r : 0];
          if (cc_ >= 0) C[cr + cc_] = acc[g][j][r];
        }
      }
    if (more) {
#pragma unroll
      for (int i = 0; i < kRowGroups; ++i) {
#pragma unroll
        for (int s = 0; s < KS; ++s) a[i][s] = an[i][s];
        r1[i] = r2[i];
      }
    }
  }
}

template <typename T, int KS, int TN, bool TR, int RV, int KV = 1>
hipError_t launch_ks_tn(int64_t batch, int M, int N, int K, const T* A, const T* B, T* C, hipStream_t s,
                        const FusedTables* f) {
  const int64_t* ra = f ? f->ra : nullptr;
  const int64_t* ca = f ? f->ca : nullptr;
  const int64_t* rb = f ? f->rb : nullptr;
  const int64_t* cb = f ? f->cb : nullptr;
  const int64_t* rc = f ? f->rc : nullptr;
  const int64_t* cc = f ? f->cc : nullptr;
  // one wave of resident workgroups over all Q (occupancy x 256 CUs), so that
  // each wave walks several row blocks with B loaded once and the next block's
  // loads in flight
  static const int resident = [] {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_gemm_rows<T, KS, TN, TR, RV, KV>, 64 * kRowWaves, 0) !=
            hipSuccess ||
        per_cu < 1) {
      (void)hipGetLastError();
      per_cu = 2;
    }
    return per_cu * 256;
  }();
  constexpr int rows = RV > 1 ? 16 * RV : 16 * row_groups<T, KS, TN>();
  const int64_t blocks = (M + rows - 1) / rows;
  const int64_t want = std::max<int64_t>(1, resident / std::max<int64_t>(batch, 1));
  const unsigned gx = static_cast<unsigned>(std::min<int64_t>((blocks + kRowWaves - 1) / kRowWaves, want));
  hipLaunchKernelGGL((k_gemm_rows<T, KS, TN, TR, RV, KV>), dim3(gx, static_cast<unsigned>(batch)), dim3(64 * kRowWaves),
                     0, s, A, B, C, M, N, K, ra, ca, rb, cb, rc, cc);
  return hipGetLastError();
}

template <typename T, int KS, bool TR>
hipError_t launch_ks(int tn, int64_t batch, int M, int N, int K, const T* A, const T* B, T* C, hipStream_t s,
                     const FusedTables* f) {
  // K-major A whose output-mode runs hold 16-byte chunks (f->vec > 1 then): row
  // vectors, binary32 only (four rows per load; binary64's pairs measured no faster)
  constexpr int VE = static_cast<int>(16 / sizeof(T));
  if constexpr (!TR && sizeof(T) == 4) {
    if (f && f->at && f->vec > 1 && M % VE == 0) {
      switch (tn) {
        case 1: return launch_ks_tn<T, KS, 1, TR, VE>(batch, M, N, K, A, B, C, s, f);
        case 2: return launch_ks_tn<T, KS, 2, TR, VE>(batch, M, N, K, A, B, C, s, f);
        case 3: return launch_ks_tn<T, KS, 3, TR, VE>(batch, M, N, K, A, B, C, s, f);
        default: return launch_ks_tn<T, KS, 4, TR, VE>(batch, M, N, K, A, B, C, s, f);
      }
    }
  }
  // A's K index contiguous in aligned runs of 16 bytes (U_al, or U's trailing
  // contracted block): K vectors, binary32 only
  if constexpr (sizeof(T) == 4 && KS % VE == 0) {
    if ((!f || !f->ra || f->a_krow) && K % VE == 0 &&
        (reinterpret_cast<uintptr_t>(A) & 15) == 0) {
      switch (tn) {
        case 1: return launch_ks_tn<T, KS, 1, TR, 1, VE>(batch, M, N, K, A, B, C, s, f);
        case 2: return launch_ks_tn<T, KS, 2, TR, 1, VE>(batch, M, N, K, A, B, C, s, f);
        case 3: return launch_ks_tn<T, KS, 3, TR, 1, VE>(batch, M, N, K, A, B, C, s, f);
        default: return launch_ks_tn<T, KS, 4, TR, 1, VE>(batch, M, N, K, A, B, C, s, f);
      }
    }
  }
  switch (tn) {
    case 1: return launch_ks_tn<T, KS, 1, TR, 1>(batch, M, N, K, A, B, C, s, f);
    case 2: return launch_ks_tn<T, KS, 2, TR, 1>(batch, M, N, K, A, B, C, s, f);
    case 3: return launch_ks_tn<T, KS, 3, TR, 1>(batch, M, N, K, A, B, C, s, f);
    default: return launch_ks_tn<T, KS, 4, TR, 1>(batch, M, N, K, A, B, C, s, f);
  }
}

template <typename T, bool TR>
hipError_t launch_tr(int64_t batch, int M, int N, int K, const T* a, const T* b, T* c, hipStream_t s,
                     const FusedTables* f) {
  const int tn = (N + 15) / 16;
  const int ks = (K + 3) / 4;
  if (ks <= 4) return launch_ks<T, 4, TR>(tn, batch, M, N, K, a, b, c, s, f);
  if (ks <= 8) return launch_ks<T, 8, TR>(tn, batch, M, N, K, a, b, c, s, f);
  if (ks <= 12) return launch_ks<T, 12, TR>(tn, batch, M, N, K, a, b, c, s, f);
  return launch_ks<T, 16, TR>(tn, batch, M, N, K, a, b, c, s, f);
}

template <typename T>
hipError_t launch_typed_rows(int64_t batch, int M, int N, int K, const void* A, const void* B, void* C,
                             hipStream_t s, const FusedTables* f) {
  const T* a = static_cast<const T*>(A);
  const T* b = static_cast<const T*>(B);
  T* c = static_cast<T*>(C);
  return f && f->c_trans ? launch_tr<T, true>(batch, M, N, K, a, b, c, s, f)
                         : launch_tr<T, false>(batch, M, N, K, a, b, c, s, f);
}

}  // namespace

// C[q] = A[q] B[q] for K <= 64 and N <= 64 (f64 when f64, else f32); f: the
// operands' offset tables (nullptr, or a null table: aligned row-major forms
// A [Q][M][K], B [Q][K][N], C [Q][M][N]) and f->c_trans, the store layout
// (same values either way).  batch <= 65535.
hipError_t launch_gemm_rows(bool f64, int64_t batch, int M, int N, int K, const void* A, const void* B, void* C,
                            hipStream_t s, const FusedTables* f) {
  if (K < 1 || K > 64 || N < 1 || N > 64 || batch < 1 || batch > 65535 || M < 1) return hipErrorInvalidValue;
  return f64 ? launch_typed_rows<double>(batch, M, N, K, A, B, C, s, f)
             : launch_typed_rows<float>(batch, M, N, K, A, B, C, s, f);
}

}  // namespace symt

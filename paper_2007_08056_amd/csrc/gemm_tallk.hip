// Long-K sector product with a small output (Alg. 2's product step where M and N
// are both at most 64 and K is long, as in a gradient with respect to a small
// tensor): C[Q] = A[Q] B[Q], f64 or f32.
//
// Such a product reads 8 (M + N) bytes per index of K for 2 M N flops: HBM
// bound, and with M, N below one 128-row tile, a tiled product would waste most
// of its MFMA work on padding.  Here workgroup (x, Q) takes the x-th range of K;
// its four waves take 16-deep groups of that range in turn and load their
// MFMA operands straight from global memory into registers (A[m][k] for the
// 16 x 4 operand of each row tile, B[k][n] likewise), one group ahead, with the
// operands' table entries two groups ahead.  Every wave accumulates the whole
// M x N output over its groups; the four waves are summed in LDS in wave order
// and the workgroup's partial goes to `part`.  k_tallk_sum then adds the
// partials of each output element in range order and writes C, so the result
// does not depend on scheduling.  Where the operands hold whole 16-deep groups
// (k_gemm_tallk_dma below) the groups stream through LDS instead, in the same
// order.  v_mfma_f64_16x16x4_f64 / v_mfma_f32_16x16x4_f32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "gemm_common.hpp"
#include "plan.hpp"

namespace symt {

namespace {

template <typename T>
struct TkMfma;
// Accumulator rows (lane l, item r; column l % 16): f64 l/16 + 4r, f32 4(l/16) + r.
template <>
struct TkMfma<double> {
  using Acc = d4;
  static __device__ __forceinline__ Acc run(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct TkMfma<float> {
  using Acc = f4;
  static __device__ __forceinline__ Acc run(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

constexpr int kTkWaves = 4;
constexpr int kTkGroup = 16;     // K indices per group (four MFMA K-steps)

// TM, TN: 16-row / 16-column tiles of the output (M <= 16 TM, N <= 16 TN).
// kc: K indices per workgroup (a multiple of kTkGroup); gridDim.x ranges per Q.
// KL (A's K index contiguous in runs of 16 or more): each lane loads A along K
// (a group's 16 K indices of one row are one 128-byte line, 4 rows per load)
// into a per-wave LDS slab, and the MFMA operands are read back from it;
// otherwise lanes load A in the MFMA operand layout (16 rows x 4 K indices).
template <typename T, int TM, int TN, bool KL>
__global__ __launch_bounds__(64 * kTkWaves) void k_gemm_tallk(
    const T* __restrict__ A, const T* __restrict__ B, T* __restrict__ part, int M, int N, int K, int kc,
    const int64_t* __restrict__ ra, const int64_t* __restrict__ ca, const int64_t* __restrict__ rb,
    const int64_t* __restrict__ cb) {
  using Acc = typename TkMfma<T>::Acc;
  constexpr int MP = 16 * TM, NP = 16 * TN;
  constexpr int LDA = kTkGroup + 1;               // slab row pitch (odd: no bank conflicts)
  constexpr int AL = KL ? 4 * TM : 1;             // A values per lane per group (K lanes)
  constexpr int AM = KL ? 1 : TM;                 // A operand registers kept across groups
  __shared__ T red[MP * NP];
  __shared__ T slab[KL ? kTkWaves : 1][KL ? MP * LDA : 1];
  const int64_t q = blockIdx.y;
  const int x = blockIdx.x;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int kq = lane >> 4;
  const int k_begin = x * kc;
  const int k_end = min(K, k_begin + kc);

  // this lane's operand rows of A (one per row tile) and columns of B (one per
  // column tile); -1 past M or N
  // (K lanes: rows (lane >> 4) + 4 j, j < 4 TM)
  constexpr int NA = KL ? 4 * TM : TM;
  int64_t arow[NA], bcol[TN];
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    const int m = KL ? (lane >> 4) + 4 * i : 16 * i + (lane & 15);
    arow[i] = m < M ? (ra ? ra[q * M + m] : (q * M + m) * static_cast<int64_t>(K)) : -1;
  }
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int n = 16 * j + (lane & 15);
    bcol[j] = n < N ? (cb ? cb[q * N + n] : static_cast<int64_t>(n)) : -1;
  }
  // table entries of the lane's four K indices of a group: A's column offset and
  // B's row offset (-1 past the range)
  // (K lanes: ak[0] is A's column offset of the lane's K index g0 + lane % 16)
  auto tables = [&](int g0, int64_t (&ak)[4], int64_t (&bk)[4]) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = g0 + 4 * u + kq;
      const bool ok = k < k_end;
      if (!KL) ak[u] = ok ? (ca ? ca[q * K + k] : static_cast<int64_t>(k)) : -1;
      bk[u] = ok ? (rb ? rb[q * K + k] : (q * K + k) * static_cast<int64_t>(N)) : -1;
    }
    if (KL) {
      const int k = g0 + (lane & 15);
      ak[0] = k < k_end ? (ca ? ca[q * K + k] : static_cast<int64_t>(k)) : -1;
    }
  };
  // the next group's operands: A (in the MFMA layout, or along K) and B
  auto operands = [&](const int64_t (&ak)[4], const int64_t (&bk)[4], T (&a)[4][AM], T (&al)[AL],
                      T (&b)[4][TN]) {
    if constexpr (KL) {
#pragma unroll
      for (int i = 0; i < AL; ++i) al[i] = ak[0] >= 0 && arow[i] >= 0 ? A[arow[i] + ak[0]] : T(0);
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int i = 0; i < TM; ++i) a[u][i] = ak[u] >= 0 && arow[i] >= 0 ? A[arow[i] + ak[u]] : T(0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int j = 0; j < TN; ++j) b[u][j] = bk[u] >= 0 && bcol[j] >= 0 ? B[bk[u] + bcol[j]] : T(0);
  };

  Acc acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = Acc{};
  const int gstep = kTkWaves * kTkGroup;
  int g = k_begin + wave * kTkGroup;
  if (g < k_end) {
    T a[4][AM], b[4][TN], an[4][AM], bn[4][TN], al[AL], aln[AL];
    int64_t ak[4], bk[4], ak2[4], bk2[4];
    tables(g, ak, bk);
    operands(ak, bk, a, al, b);
    if (g + gstep < k_end) tables(g + gstep, ak, bk);
    for (; g < k_end; g += gstep) {
      const bool more = g + gstep < k_end;
      if (g + 2 * gstep < k_end) tables(g + 2 * gstep, ak2, bk2);
      if (more) operands(ak, bk, an, aln, bn);
      if constexpr (KL) {
        // this group's A through the wave's slab into the MFMA layout
        T* sl = slab[wave];
#pragma unroll
        for (int i = 0; i < AL; ++i) sl[((lane >> 4) + 4 * i) * LDA + (lane & 15)] = al[i];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int i = 0; i < TM; ++i) {
            const T av = sl[(16 * i + (lane & 15)) * LDA + 4 * u + kq];
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = TkMfma<T>::run(av, b[u][j], acc[i][j]);
          }
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = TkMfma<T>::run(a[u][i], b[u][j], acc[i][j]);
      }
      if (more) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if constexpr (!KL) {
#pragma unroll
            for (int i = 0; i < TM; ++i) a[u][i] = an[u][i];
          }
#pragma unroll
          for (int j = 0; j < TN; ++j) b[u][j] = bn[u][j];
          ak[u] = ak2[u];
          bk[u] = bk2[u];
        }
        if constexpr (KL) {
#pragma unroll
          for (int i = 0; i < AL; ++i) al[i] = aln[i];
        }
      }
    }
  }
  // the four waves' sums in wave order, then the workgroup's partial [m][n]
  for (int w = 0; w < kTkWaves; ++w) {
    if (wave == w) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int e = (16 * i + TkMfma<T>::row(lane, r)) * NP + 16 * j + (lane & 15);
            red[e] = w == 0 ? acc[i][j][r] : red[e] + acc[i][j][r];
          }
    }
    __syncthreads();
  }
  T* pw = part + (q * gridDim.x + x) * static_cast<int64_t>(M) * N;
  for (int e = static_cast<int>(threadIdx.x); e < M * N; e += 64 * kTkWaves) {
    const int m = e / N, n = e - (e / N) * N;
    pw[e] = red[m * NP + n];
  }
}

// Global-to-LDS variant, where every 16-deep group of K lies in one contiguous
// run of A's rows and one affine run of B's rows, and B's columns come in whole
// 16-byte chunks: each wave streams its own groups (the same groups, in the same
// order, as above, so both variants give the same bits) through a private
// S-stage LDS ring with global_load_lds_dwordx4 (A: the group's 16 K values of
// each row, 128 or 64 bytes; B: the group's 16 rows in 16-byte chunks), so a
// group costs no staging registers and S - 1 groups stay in flight per wave.
// The waves never wait on each other until the final sum.
// LDS slots: A (r, p) holds chunk p ^ tk_aswz(r) of row r, B (k, p) holds chunk
// p ^ tk_bswz(k); with these the MFMA operand reads hit distinct banks.  Rows
// past M and chunks past N are clamped on load and never stored.
template <typename T>
__device__ __forceinline__ int tk_aswz(int r) {
  if constexpr (sizeof(T) == 8) return (r >> 1) & 7;     // 8 chunks per 128-byte row
  else return (r >> 2) & 3;                              // 4 chunks per 64-byte row
}
template <typename T, int NP>
__device__ __forceinline__ int tk_bswz(int k) {
  constexpr int row_bytes = NP * static_cast<int>(sizeof(T));
  if constexpr (sizeof(T) == 8) return row_bytes % 256 == 0 ? (k & 1) << 3 : 0;
  else if constexpr (row_bytes % 256 == 0) return (k & 3) << 2;
  else if constexpr (row_bytes % 256 == 128) return ((k >> 1) & 1) << 2;
  else return 0;
}

template <typename T, int TM, int TN>
struct TkDma {
  static constexpr int E = static_cast<int>(sizeof(T));
  static constexpr int VE = 16 / E;                        // elements per 16-byte chunk
  static constexpr int GK = kTkGroup;                      // K indices per group
  static constexpr int CPR = GK / VE;                      // A chunks per row and group
  static constexpr int MP = 16 * TM, NP = 16 * TN;
  static constexpr int BCH = NP / VE;                      // chunks per B row
  static constexpr int A_LOADS = MP * CPR / 64, B_LOADS = GK * BCH / 64;
  static constexpr int LOADS = A_LOADS + B_LOADS;
  static constexpr int A_BYTES = MP * GK * E;
  static constexpr int STAGE = A_BYTES + GK * NP * E;
  static constexpr int LDS = 160 * 1024;
  static constexpr int S = LDS / (kTkWaves * STAGE) >= 4 ? 4 : LDS / (kTkWaves * STAGE) >= 3 ? 3 : 2;
  static_assert(A_LOADS * 64 == MP * CPR && B_LOADS * 64 == GK * BCH, "loads must fill whole waves");
  static_assert(kTkWaves * S * STAGE <= LDS && (S - 1) * LOADS < 64, "ring");
  static_assert(MP * NP * E <= kTkWaves * S * STAGE, "sum space");
};

// vmcnt <= n LOADS-sized groups of loads (n < 4)
template <int LOADS>
__device__ __forceinline__ void tk_wait_groups(int n) {
  switch (n) {
    case 0: wait_vmcnt<0>(); break;
    case 1: wait_vmcnt<LOADS>(); break;
    case 2: wait_vmcnt<2 * LOADS < 64 ? 2 * LOADS : 0>(); break;
    default: wait_vmcnt<3 * LOADS < 64 ? 3 * LOADS : 0>(); break;
  }
}

template <typename T, int TM, int TN>
__global__ __launch_bounds__(64 * kTkWaves) void k_gemm_tallk_dma(
    const T* __restrict__ A, const T* __restrict__ B, T* __restrict__ part, int M, int N, int K, int kc,
    const int64_t* __restrict__ ra, const int64_t* __restrict__ ca, const int64_t* __restrict__ rb,
    const int64_t* __restrict__ cb, int64_t ldb) {
  using D = TkDma<T, TM, TN>;
  using Acc = typename TkMfma<T>::Acc;
  constexpr int VE = D::VE, GK = D::GK, CPR = D::CPR, MP = D::MP, NP = D::NP, BCH = D::BCH, S = D::S;
  constexpr int A_LOADS = D::A_LOADS, B_LOADS = D::B_LOADS, LOADS = D::LOADS, STAGE = D::STAGE;
  constexpr int A_BYTES = D::A_BYTES;
  __shared__ __attribute__((aligned(16))) char smem[kTkWaves * S * STAGE];
  const int64_t q = blockIdx.y;
  const int x = blockIdx.x;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int k_begin = x * kc;
  const int k_end = min(K, k_begin + kc);
  char* ring = smem + wave * S * STAGE;

  // this lane's load sources, fixed across groups: A row base + chunk, B row k of
  // a group + column chunk
  int64_t a_src[A_LOADS], b_src[B_LOADS];
#pragma unroll
  for (int i = 0; i < A_LOADS; ++i) {
    const int slot = i * 64 + lane;
    const int r = slot / CPR, c = (slot % CPR) ^ tk_aswz<T>(r);
    const int gr = min(r, M - 1);
    a_src[i] = (ra ? ra[q * M + gr] : (q * M + gr) * static_cast<int64_t>(K)) + c * VE;
  }
#pragma unroll
  for (int i = 0; i < B_LOADS; ++i) {
    const int slot = i * 64 + lane;
    const int k = slot / BCH, c = (slot % BCH) ^ tk_bswz<T, NP>(k);
    const int gn = min(c * VE, N - VE);
    b_src[i] = k * ldb + (cb ? cb[q * N + gn] : static_cast<int64_t>(gn));
  }
  // a group's A column offset and B row offset (wave-uniform)
  auto acol_of = [&](int g) { return ca ? ca[q * K + g] : static_cast<int64_t>(g); };
  auto brow_of = [&](int g) { return rb ? rb[q * K + g] : (q * K + g) * static_cast<int64_t>(N); };
  auto issue = [&](int stage, int64_t acol, int64_t brow) {
    char* base = ring + stage * STAGE;
#pragma unroll
    for (int i = 0; i < A_LOADS; ++i) lds_dma16(A + a_src[i] + acol, base + i * 1024);
#pragma unroll
    for (int i = 0; i < B_LOADS; ++i) lds_dma16(B + b_src[i] + brow, base + A_BYTES + i * 1024);
  };

  Acc acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = Acc{};
  const int g0 = k_begin + wave * GK;
  const int gstep = kTkWaves * GK;
  const int ng = g0 < k_end ? (k_end - g0 + gstep - 1) / gstep : 0;
#pragma unroll
  for (int s = 0; s < S - 1; ++s)
    if (s < ng) issue(s, acol_of(g0 + s * gstep), brow_of(g0 + s * gstep));
  // table entries of the next group to issue, fetched one iteration ahead
  int64_t acol_n = 0, brow_n = 0;
  if (S - 1 < ng) {
    acol_n = acol_of(g0 + (S - 1) * gstep);
    brow_n = brow_of(g0 + (S - 1) * gstep);
  }
  for (int it = 0; it < ng; ++it) {
    // the stage refilled next was read by the previous group's operand loads
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0), vmcnt and expcnt untouched
    const int nxt = it + S - 1;
    if (nxt < ng) {
      issue(nxt % S, acol_n, brow_n);
      if (nxt + 1 < ng) {
        acol_n = acol_of(g0 + (nxt + 1) * gstep);
        brow_n = brow_of(g0 + (nxt + 1) * gstep);
      }
    }
    tk_wait_groups<LOADS>(min(ng - 1, nxt) - it);
    asm volatile("" ::: "memory");        // the operand reads below stay after the wait
    const char* base = ring + (it % S) * STAGE;
    const T* As = reinterpret_cast<const T*>(base);
    const T* Bs = reinterpret_cast<const T*>(base + A_BYTES);
#pragma unroll
    for (int kk = 0; kk < GK; kk += 4) {
      const int k = kk + (lane >> 4);
      T a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int m = 16 * i + (lane & 15);
        a[i] = As[m * GK + ((k / VE) ^ tk_aswz<T>(m)) * VE + k % VE];
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int n = 16 * j + (lane & 15);
        b[j] = Bs[k * NP + ((n / VE) ^ tk_bswz<T, NP>(k)) * VE + n % VE];
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = TkMfma<T>::run(a[i], b[j], acc[i][j]);
    }
  }
  // the four waves' sums in wave order (over the rings, once every wave is done
  // with its own), then the workgroup's partial [m][n]
  T* red = reinterpret_cast<T*>(smem);
  __syncthreads();
  for (int w = 0; w < kTkWaves; ++w) {
    if (wave == w) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int e = (16 * i + TkMfma<T>::row(lane, r)) * NP + 16 * j + (lane & 15);
            red[e] = w == 0 ? acc[i][j][r] : red[e] + acc[i][j][r];
          }
    }
    __syncthreads();
  }
  T* pw = part + (q * gridDim.x + x) * static_cast<int64_t>(M) * N;
  for (int e = static_cast<int>(threadIdx.x); e < M * N; e += 64 * kTkWaves) {
    const int m = e / N, n = e - (e / N) * N;
    pw[e] = red[m * NP + n];
  }
}

// C = the sum over ranges, in range order, of the partials (one thread per
// output element; grid (elements / 256, Q)).
template <typename T>
__global__ __launch_bounds__(256) void k_tallk_sum(const T* __restrict__ part, T* __restrict__ C, int M, int N,
                                                   int ranges, const int64_t* __restrict__ rc,
                                                   const int64_t* __restrict__ cc) {
  const int64_t q = blockIdx.y;
  const int e = static_cast<int>(blockIdx.x) * 256 + static_cast<int>(threadIdx.x);
  if (e >= M * N) return;
  const int64_t mn = static_cast<int64_t>(M) * N;
  const T* p = part + q * ranges * mn + e;
  T acc = T(0);
#pragma unroll 8
  for (int x = 0; x < ranges; ++x) acc += p[x * mn];
  const int m = e / N, n = e - (e / N) * N;
  const int64_t off = rc ? rc[q * M + m] + cc[q * N + n] : (q * M + m) * static_cast<int64_t>(N) + n;
  C[off] = acc;
}

template <typename T, int TM, int TN>
hipError_t launch_mn(int64_t batch, int M, int N, int K, const T* A, const T* B, T* C, hipStream_t s,
                     const FusedTables* f, T* part, int ranges, int kc) {
  // A's K index contiguous (the aligned form, or a hint from the plan): loads
  // along K, binary32 only (binary64 would hold one wave per SIMD: 263 registers)
  const bool kl = sizeof(T) == 4 && (!f || !f->ra || f->a_klanes);
  const int64_t* ra = f ? f->ra : nullptr;
  const int64_t* ca = f ? f->ca : nullptr;
  const int64_t* rb = f ? f->rb : nullptr;
  const int64_t* cb = f ? f->cb : nullptr;
  const int64_t* rc = f ? f->rc : nullptr;
  const int64_t* cc = f ? f->cc : nullptr;
  const dim3 grid(static_cast<unsigned>(ranges), static_cast<unsigned>(batch));
  // whole 16-deep groups of K in A's runs and B's affine K-steps, 16-byte
  // chunks of B's columns, 16-byte aligned operands: the global-to-LDS variant
  constexpr int GK = TkDma<T, TM, TN>::GK, VE = TkDma<T, TM, TN>::VE;
  const bool dma = K % GK == 0 && N % VE == 0 &&
                   ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B)) & 15) == 0 &&
                   (!f || (!f->ra && !f->rb) || f->k_groups);
  if (dma) {
    hipLaunchKernelGGL((k_gemm_tallk_dma<T, TM, TN>), grid, dim3(64 * kTkWaves), 0, s, A, B, part, M, N, K, kc,
                       ra, ca, rb, cb, f && f->rb ? f->ldb : static_cast<int64_t>(N));
  } else if (kl)
    hipLaunchKernelGGL((k_gemm_tallk<T, TM, TN, true>), grid, dim3(64 * kTkWaves), 0, s, A, B, part, M, N, K, kc,
                       ra, ca, rb, cb);
  else
    hipLaunchKernelGGL((k_gemm_tallk<T, TM, TN, false>), grid, dim3(64 * kTkWaves), 0, s, A, B, part, M, N, K,
                       kc, ra, ca, rb, cb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_tallk_sum<T>), dim3(static_cast<unsigned>((M * N + 255) / 256), static_cast<unsigned>(batch)),
                     dim3(256), 0, s, part, C, M, N, ranges, rc, cc);
  return hipGetLastError();
}

template <typename T, int TM>
hipError_t launch_m(int tn, int64_t batch, int M, int N, int K, const T* A, const T* B, T* C, hipStream_t s,
                    const FusedTables* f, T* part, int ranges, int kc) {
  switch (tn) {
    case 1: return launch_mn<T, TM, 1>(batch, M, N, K, A, B, C, s, f, part, ranges, kc);
    case 2: return launch_mn<T, TM, 2>(batch, M, N, K, A, B, C, s, f, part, ranges, kc);
    case 3: return launch_mn<T, TM, 3>(batch, M, N, K, A, B, C, s, f, part, ranges, kc);
    default: return launch_mn<T, TM, 4>(batch, M, N, K, A, B, C, s, f, part, ranges, kc);
  }
}

template <typename T>
hipError_t launch_typed_tallk(int64_t batch, int M, int N, int K, const void* A, const void* B, void* C,
                              hipStream_t s, const FusedTables* f, void* part, int ranges) {
  const T* a = static_cast<const T*>(A);
  const T* b = static_cast<const T*>(B);
  T* c = static_cast<T*>(C);
  T* pt = static_cast<T*>(part);
  const int kc = tallk_range(K, ranges);
  const int tm = (M + 15) / 16, tn = (N + 15) / 16;
  switch (tm) {
    case 1: return launch_m<T, 1>(tn, batch, M, N, K, a, b, c, s, f, pt, ranges, kc);
    case 2: return launch_m<T, 2>(tn, batch, M, N, K, a, b, c, s, f, pt, ranges, kc);
    case 3: return launch_m<T, 3>(tn, batch, M, N, K, a, b, c, s, f, pt, ranges, kc);
    default: return launch_m<T, 4>(tn, batch, M, N, K, a, b, c, s, f, pt, ranges, kc);
  }
}

}  // namespace

// C[q] = A[q] B[q] for M, N <= 64 (f64 when f64, else f32) over `ranges` ranges
// of K per slice (tallk_ranges); `part` holds batch * ranges * M * N partials.
// f: the operands' offset tables (nullptr or null tables: aligned row-major
// A [Q][M][K], B [Q][K][N], C [Q][M][N]).  batch <= 65535.
hipError_t launch_gemm_tallk(bool f64, int64_t batch, int M, int N, int K, const void* A, const void* B, void* C,
                             hipStream_t s, const FusedTables* f, void* part, int ranges) {
  if (M < 1 || M > 64 || N < 1 || N > 64 || K < 1 || batch < 1 || batch > 65535 || ranges < 1 || !part)
    return hipErrorInvalidValue;
  return f64 ? launch_typed_tallk<double>(batch, M, N, K, A, B, C, s, f, part, ranges)
             : launch_typed_tallk<float>(batch, M, N, K, A, B, C, s, f, part, ranges);
}

}  // namespace symt

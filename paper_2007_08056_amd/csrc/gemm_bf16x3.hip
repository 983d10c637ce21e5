// Split-bf16 sector product on wide global-to-LDS tiles (Alg. 2's product step
// in the split-bfloat16 precision form): C[Q] = A[Q] B[Q] with A = Ahi + Alo and
// B = Bhi + Blo given as bf16 planes (A [Q][M][K], B [Q][N][K], K fastest), C as
// binary64 (aligned W, or W's standard form through its offset tables).
//
// Each workgroup owns a BM x BN output tile with WM x WN waves; a wave owns a
// (BM/WM) x (BN/WN) block of 16 x 16 MFMA tiles (v_mfma_f32_16x16x32_bf16) and
// keeps ONE binary32 accumulator per output element, into which it adds
// Ahi*Bhi, Ahi*Blo and Alo*Bhi.  One accumulator (rather than one for hi*hi and
// one for the cross terms) halves the accumulator registers, so a wave can hold
// a 128 x 64 block in half a SIMD's registers: the 256 x 256 tile runs eight
// waves, two per SIMD, so that one wave's MFMAs cover the other's wait at the
// K-step barrier and on its fragment reads (the four-wave form, one 128 x 128
// block per wave, left the matrix pipes idle there: 0.53 against 0.59 of the
// bf16 peak on the Z_16 ladder's product).  The accumulators live in AGPRs, so
// this file is compiled without the VGPR-form flag of the other product kernels.
//
// K-steps are 32 deep (one MFMA); each stage of the LDS ring holds one K-step
// of the four planes, loaded with global_load_lds (16 bytes per lane) into
// rows of 64 bytes whose four chunks are XOR-swizzled by ((row >> 1) & 3), so
// the fragment reads of 8 consecutive rows fall on distinct banks.  Rows past M
// or N are clamped on load and never stored; K must be a multiple of 32.
//
// IL: the planes interleaved by K-steps ([Q][row][K / 32][hi 32 | lo 32], the
// layout the contraction's transforms write for these tiles).  A row's K-step
// is then one whole 128-byte line instead of two half lines 32 K-steps of
// planes apart, which halves the lines each workgroup has in flight per K-step
// (the kernel is bound by those line requests, not by HBM bytes).  The stage
// keeps each row's 128 bytes together, its eight 16-byte chunks XOR-swizzled
// by (row & 7).
//
// FA: A read in place from U's standard form (binary32, runs of 4 along K at
// 16-byte aligned offsets ra(Q, m) + ca(Q, k)) and split into hi/lo when the
// fragments are read, as the transforms split it (bf16_split): the stage holds
// each row's 32 binary32 values (128 bytes, the interleaved planes' size), its
// eight 16-byte chunks XOR-swizzled by (row & 7); a K-step's column offsets are
// fetched one step ahead of its loads.  This drops the pass that would put U on
// planes (a read and a write of U) for 24 conversions and subtractions per
// fragment (the 64 x 128 wave blocks read half the A fragments of 128 x 64).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>
#include <type_traits>

#include "bf16_split.hpp"
#include "gemm_common.hpp"
#include "plan.hpp"

namespace symt {

namespace {

typedef float fv4 __attribute__((ext_vector_type(4)));
typedef float fv8 __attribute__((ext_vector_type(8)));
typedef uint32_t uv4 __attribute__((ext_vector_type(4)));

// bf16_split of eight binary32 values at once: hi = bf16(x), lo = bf16(x - hi),
// each by the hardware conversion that bf16_rne is (paired, round to nearest even).
__device__ __forceinline__ void split8(fv4 x0, fv4 x1, bf8& hi, bf8& lo) {
  const fv8 x = {x0[0], x0[1], x0[2], x0[3], x1[0], x1[1], x1[2], x1[3]};
  hi = __builtin_convertvector(x, bf8);
  const uv4 hb = __builtin_bit_cast(uv4, hi);
  fv8 hf;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    hf[2 * j] = __uint_as_float(hb[j] << 16);
    hf[2 * j + 1] = __uint_as_float(hb[j] & 0xFFFF0000u);
  }
  lo = __builtin_convertvector(x - hf, bf8);
}

template <int BM, int BN, int WM, int WN, int S, bool FC, typename TC, bool IL, bool FA>
__global__ __launch_bounds__(64 * WM * WN, 1) void k_bf16x3_wide(
    const uint16_t* __restrict__ Ahi, const uint16_t* __restrict__ Alo, const uint16_t* __restrict__ Bhi,
    const uint16_t* __restrict__ Blo, TC* __restrict__ C, int M, int N, int K, int tiles_m, int tiles_n,
    int64_t ntiles, const int64_t* __restrict__ rc, const int64_t* __restrict__ cc, int group_m,
    const float* __restrict__ U, const int64_t* __restrict__ ra, const int64_t* __restrict__ ca) {
  constexpr int NT = 64 * WM * WN;
  constexpr int BK = 32;
  constexpr int TM = BM / WM / 16;
  constexpr int TN = BN / WN / 16;
  constexpr int A_LOADS = BM * 8 / NT;            // 16-byte chunks of both A planes per thread
  constexpr int B_LOADS = BN * 8 / NT;
  constexpr int PA = BM * 64, PB = BN * 64;       // bytes per plane per stage
  constexpr int STAGE = 2 * PA + 2 * PB;
  static_assert(TM * WM * 16 == BM && TN * WN * 16 == BN, "tile shape");
  static_assert(A_LOADS * NT == BM * 8 && B_LOADS * NT == BN * 8, "loads must divide evenly");
  static_assert(S >= 2 && S * STAGE <= 160 * 1024, "LDS ring");
  static_assert(FC || std::is_same<TC, double>::value, "aligned W is binary64");
  static_assert(!FA || (IL && S == 2), "A in place: interleaved B planes and two stages");
  __shared__ __attribute__((aligned(1024))) char smem[S * STAGE];

  const int64_t tile = xcd_remap(blockIdx.x, ntiles);
  int64_t q;
  int tm, tn;
  tile_coords(tile, tiles_m, tiles_n, q, tm, tn, group_m);
  const int m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm0 = (wave / WN) * (BM / WM);
  const int wn0 = (wave % WN) * (BN / WN);
  const int64_t offA = q * static_cast<int64_t>(M) * K * (IL ? 2 : 1);
  const int64_t offB = q * static_cast<int64_t>(N) * K * (IL ? 2 : 1);

  // Load slot s = tid + i * NT covers [plane][row][chunk]; LDS position c of row
  // r holds global chunk c ^ ((r >> 1) & 3).  IL: slot s covers [row][chunk of
  // 8] and position c of row r holds chunk c ^ (r & 7) of the row's K-step
  // (chunks 0-3 hi, 4-7 lo).
  const uint16_t* a_src[A_LOADS];
  // FA: U's row offset and the in-step K offset (4 x chunk) of each load slot,
  // and the column offsets of the next K-step to issue
  const float* a_row[A_LOADS];
  int a_k[A_LOADS];
  int64_t a_col[A_LOADS];
#pragma unroll
  for (int i = 0; i < A_LOADS; ++i) {
    const int slot = tid + i * NT;
    if constexpr (FA) {
      const int r = slot >> 3;
      a_row[i] = U + ra[q * M + min(m0 + r, M - 1)];
      a_k[i] = ((slot & 7) ^ (r & 7)) * 4;
    } else if constexpr (IL) {
      const int r = slot >> 3;
      a_src[i] = Ahi + offA + static_cast<int64_t>(min(m0 + r, M - 1)) * 2 * K + ((slot & 7) ^ (r & 7)) * 8;
    } else {
      const int plane = slot / (BM * 4);
      const int rem = slot - plane * (BM * 4);
      const int r = rem >> 2, c = rem & 3;
      const int gr = min(m0 + r, M - 1);
      a_src[i] = (plane ? Alo : Ahi) + offA + static_cast<int64_t>(gr) * K + (c ^ ((r >> 1) & 3)) * 8;
    }
  }
  const uint16_t* b_src[B_LOADS];
#pragma unroll
  for (int i = 0; i < B_LOADS; ++i) {
    const int slot = tid + i * NT;
    if constexpr (IL) {
      const int r = slot >> 3;
      b_src[i] = Bhi + offB + static_cast<int64_t>(min(n0 + r, N - 1)) * 2 * K + ((slot & 7) ^ (r & 7)) * 8;
    } else {
      const int plane = slot / (BN * 4);
      const int rem = slot - plane * (BN * 4);
      const int r = rem >> 2, c = rem & 3;
      const int gr = min(n0 + r, N - 1);
      b_src[i] = (plane ? Blo : Bhi) + offB + static_cast<int64_t>(gr) * K + (c ^ ((r >> 1) & 3)) * 8;
    }
  }
  auto fetch_cols = [&](int kt) {
#pragma unroll
    for (int i = 0; i < A_LOADS; ++i) a_col[i] = ca[q * K + kt * BK + a_k[i]];
  };
  auto issue = [&](int kt, int stage) {
    const int k0 = kt * (IL ? 2 * BK : BK);
    char* base = smem + stage * STAGE;
#pragma unroll
    for (int i = 0; i < A_LOADS; ++i) {
      if constexpr (FA) lds_dma16(a_row[i] + a_col[i], base + (i * NT + wave * 64) * 16);
      else lds_dma16(a_src[i] + k0, base + (i * NT + wave * 64) * 16);
    }
#pragma unroll
    for (int i = 0; i < B_LOADS; ++i) lds_dma16(b_src[i] + k0, base + 2 * PA + (i * NT + wave * 64) * 16);
  };

  f4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f4{};

  const int nk = K / BK;
  const int kc = lane >> 4;                       // operand chunk: k = 8 * kc .. 8 * kc + 7
  if constexpr (FA) {
    // (two stages: the loop's wait for nothing outstanding also covers the
    // column offsets fetched one step ahead)
    if (nk > 0) {
      fetch_cols(0);
      wait_vmcnt<0>();
      issue(0, 0);
      if (nk > 1) fetch_cols(1);
    }
  } else {
#pragma unroll
    for (int s = 0; s < S - 1; ++s)
      if (s < nk) issue(s, s);
  }
  for (int kt = 0; kt < nk; ++kt) {
    // step kt has landed once at most (S - 2) later steps' loads are outstanding
    if (kt + S - 2 < nk) wait_vmcnt<(S - 2) * (A_LOADS + B_LOADS)>();
    else wait_vmcnt<0>();
    // a plain barrier: the wait above covers this wave's loads of step kt, and
    // every wave has finished reading the stage that the next issue overwrites
    asm volatile("s_barrier" ::: "memory");
    if (kt + S - 1 < nk) {
      issue(kt + S - 1, (kt + S - 1) % S);
      if constexpr (FA)
        if (kt + 2 < nk) fetch_cols(kt + 2);
    }
    const char* base = smem + (kt % S) * STAGE;
    bf8 ah[TM], al[TM];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const int r = wm0 + i * 16 + (lane & 15);
      if constexpr (FA) {
        // K 8 kc .. 8 kc + 7 of row r: chunks 2 kc and 2 kc + 1
        const fv4 x0 = *reinterpret_cast<const fv4*>(base + r * 128 + (((2 * kc) ^ (r & 7)) << 4));
        const fv4 x1 = *reinterpret_cast<const fv4*>(base + r * 128 + (((2 * kc + 1) ^ (r & 7)) << 4));
        split8(x0, x1, ah[i], al[i]);
      } else {
        const int off = IL ? r * 128 + ((kc ^ (r & 7)) << 4) : r * 64 + ((kc ^ ((r >> 1) & 3)) << 4);
        const int off_lo = IL ? r * 128 + (((4 + kc) ^ (r & 7)) << 4) : PA + off;
        ah[i] = *reinterpret_cast<const bf8*>(base + off);
        al[i] = *reinterpret_cast<const bf8*>(base + off_lo);
      }
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int r = wn0 + j * 16 + (lane & 15);
      const int off = 2 * PA + (IL ? r * 128 + ((kc ^ (r & 7)) << 4) : r * 64 + ((kc ^ ((r >> 1) & 3)) << 4));
      const int off_lo = IL ? 2 * PA + r * 128 + (((4 + kc) ^ (r & 7)) << 4) : PB + off;
      const bf8 bh = *reinterpret_cast<const bf8*>(base + off);
      const bf8 bl = *reinterpret_cast<const bf8*>(base + off_lo);
      // consecutive MFMAs update different accumulators (no dependent back-to-back pairs)
#pragma unroll
      for (int i = 0; i < TM; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh, acc[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < TM; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl, acc[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < TM; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh, acc[i][j], 0, 0, 0);
    }
  }

  // 16x16x32 bf16 accumulator layout: lane l, item r holds row 4 (l / 16) + r, column l % 16
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
          Cq[crow + ccol] = static_cast<TC>(acc[i][j][r]);
        }
      }
  }
}

template <int BM, int BN, int WM, int WN, int S, bool IL, bool FA = false>
hipError_t launch_wide(int64_t batch, int M, int N, int K, const void* A, const void* B, void* C, hipStream_t s,
                       int64_t pa, int64_t pb, const int64_t* rc, const int64_t* cc, int c_bytes,
                       const int64_t* ra = nullptr, const int64_t* ca = nullptr) {
  const int tiles_m = (M + BM - 1) / BM, tiles_n = (N + BN - 1) / BN;
  const int64_t ntiles = batch * tiles_m * tiles_n;
  const dim3 grid(static_cast<unsigned>(ntiles)), block(64 * WM * WN);
  const uint16_t* a = FA ? nullptr : static_cast<const uint16_t*>(A);
  const float* u = FA ? static_cast<const float*>(A) : nullptr;
  const uint16_t* b = static_cast<const uint16_t*>(B);
  // M-panels per group of the tile order (each XCD runs a contiguous range of
  // tiles, so the workgroups in flight on one XCD are group_m M-panels by a few
  // N-tiles); 8 measured best on the Z_16 ladder (4 to 64 tried).
  // SYMT_GEMM_GROUP_M overrides it (tuning only).
  const char* gm_env = std::getenv("SYMT_GEMM_GROUP_M");
  int gm = gm_env ? std::atoi(gm_env) : 8;
  if (gm < 1) gm = 1;
  if (rc && c_bytes == 4)
    hipLaunchKernelGGL((k_bf16x3_wide<BM, BN, WM, WN, S, true, float, IL, FA>), grid, block, 0, s, a, a + pa, b, b + pb,
                       static_cast<float*>(C), M, N, K, tiles_m, tiles_n, ntiles, rc, cc, gm, u, ra, ca);
  else if (rc)
    hipLaunchKernelGGL((k_bf16x3_wide<BM, BN, WM, WN, S, true, double, IL, FA>), grid, block, 0, s, a, a + pa, b, b + pb,
                       static_cast<double*>(C), M, N, K, tiles_m, tiles_n, ntiles, rc, cc, gm, u, ra, ca);
  else if constexpr (!FA)
    hipLaunchKernelGGL((k_bf16x3_wide<BM, BN, WM, WN, S, false, double, IL, false>), grid, block, 0, s, a, a + pa, b,
                       b + pb, static_cast<double*>(C), M, N, K, tiles_m, tiles_n, ntiles, rc, cc, gm, u, ra, ca);
  else
    return hipErrorInvalidValue;   // A in place writes W in place
  return hipGetLastError();
}

}  // namespace

// Wide split-bf16 tiles: 0 = 256 x 256 (8 waves of 128 x 64, two LDS stages),
// 1 = 256 x 128 (4 waves of 128 x 64, three stages).  pa / pb: elements from
// each hi plane to its lo plane (unused with il); rc / cc: W's offset tables
// (nullptr: C is the aligned W, binary64); il: planes interleaved by K-steps;
// ra / ca (with il, variant 0 and W's tables): A is U's standard form in
// binary32, read through these tables (FA above).  Needs K % 32 == 0 and
// 16-byte aligned planes.
hipError_t launch_bf16x3_wide(int variant, int64_t batch, int M, int N, int K, const void* A, const void* B,
                              void* C, hipStream_t s, int64_t pa, int64_t pb, const int64_t* rc,
                              const int64_t* cc, int c_bytes, bool il, const int64_t* ra, const int64_t* ca) {
  // A in place (binary32 U through ra / ca): the 256 x 256 tile with 64 x 128 wave blocks
  if (ra && ca) {
    if (!il || variant != 0 || !rc) return hipErrorInvalidValue;
    return launch_wide<256, 256, 4, 2, 2, true, true>(batch, M, N, K, A, B, C, s, pa, pb, rc, cc, c_bytes, ra, ca);
  }
  if (il)
    return variant == 1 ? launch_wide<256, 128, 2, 2, 3, true>(batch, M, N, K, A, B, C, s, pa, pb, rc, cc, c_bytes)
                        : launch_wide<256, 256, 2, 4, 2, true>(batch, M, N, K, A, B, C, s, pa, pb, rc, cc, c_bytes);
  if (variant == 1) return launch_wide<256, 128, 2, 2, 3, false>(batch, M, N, K, A, B, C, s, pa, pb, rc, cc, c_bytes);
  return launch_wide<256, 256, 2, 4, 2, false>(batch, M, N, K, A, B, C, s, pa, pb, rc, cc, c_bytes);
}

}  // namespace symt

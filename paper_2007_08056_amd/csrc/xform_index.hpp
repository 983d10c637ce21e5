// Index arithmetic of the reduced-form transforms, shared by the kernels and
// host-side checks: group operations on flattened elements, the implicit
// sector of a sector group (one generalized Kronecker delta of Alg. 2), and
// the two base offsets of one block in the standard and aligned layouts.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.hpp"

namespace symt {

__host__ __device__ inline int dg_add(const GroupDesc& g, int a, int b) {
  if (g.nf == 1) {
    const int s = a + b;
    return s >= g.size ? s - g.size : s;
  }
  int r = 0, mul = 1;
  for (int f = g.nf - 1; f >= 0; --f) {
    const int o = g.ord[f];
    const int da = a % o, db = b % o;
    a /= o;
    b /= o;
    const int s = da + db;
    r += (s >= o ? s - o : s) * mul;
    mul *= o;
  }
  return r;
}

__host__ __device__ inline int dg_neg(const GroupDesc& g, int a) {
  if (g.nf == 1) return a == 0 ? 0 : g.size - a;
  int r = 0, mul = 1;
  for (int f = g.nf - 1; f >= 0; --f) {
    const int o = g.ord[f];
    const int da = a % o;
    a /= o;
    r += (da == 0 ? 0 : o - da) * mul;
    mul *= o;
  }
  return r;
}

__host__ __device__ inline int dg_times(const GroupDesc& g, int c, int a) {
  return c >= 0 ? a : dg_neg(g, a);
}

// Sector labels of one group's modes: the stored ones are the digits of
// `digits` (mixed radix over the members' sector counts, first most
// significant); the last one solves the group's delta.  The deltas hold on
// charges: with charge tables `chg` ([mode][label -> charge | charge -> label]
// [|G|], nullptr for identity) the stored labels are mapped to charges and the
// solved charge back to a label.  A subgroup member (H < |G| sectors,
// coefficient +-|G|/H; cyclic groups only) adds mag * label; as the last
// member its equation s mag x == r has a solution only when mag divides r.
// Returns false when the block does not exist.
template <typename I>
__host__ __device__ inline bool fill_sectors(const GroupDesc& g, const SectorGroup& sg,
                                             I digits, int q, int* S, const int32_t* chg) {
  if (sg.count == 0) return true;   // an empty group only pins Q
  int acc = 0;
  for (int i = sg.count - 2; i >= 0; --i) {
    const int d = static_cast<int>(digits % sg.rad[i]);
    digits /= sg.rad[i];
    S[sg.pos[i]] = d;
    int c = chg ? chg[(2 * sg.pos[i]) * g.size + d] : d;
    if (sg.mag[i] != 1) c = (sg.mag[i] * c) % g.size;
    acc = dg_add(g, acc, dg_times(g, sg.coef[i], c));
  }
  const int rhs = dg_add(g, dg_times(g, sg.alpha, q), sg.beta);
  const int n = sg.count - 1;
  const int last = sg.pos[n];
  const int r = dg_add(g, rhs, dg_neg(g, acc));
  if (sg.mag[n] != 1) {
    if (r % sg.mag[n] != 0) return false;
    const int x = r / sg.mag[n];
    S[last] = sg.coef[n] >= 0 || x == 0 ? x : sg.rad[n] - x;
    return true;
  }
  const int c = dg_times(g, sg.coef[n], r);
  S[last] = chg ? chg[(2 * last + 1) * g.size + c] : c;
  return true;
}

// Aligned block index -> (standard-form element offset, aligned element
// offset); false when the block does not exist (its aligned block is zero).
// (I: the index type of the block arithmetic, 32-bit where the block count fits)
template <typename I>
__host__ __device__ inline bool block_bases_t(const XformParams& p, I blk, int64_t& std_base, int64_t& al_base) {
  const I gc = static_cast<I>(p.gpow_col), gr = static_cast<I>(p.gpow_row);
  const I cs = blk % gc;
  const I t = blk / gc;
  const I rs = t % gr;
  const I slice = t / gr;
  const int q = p.q0 + p.q_step * static_cast<int>(slice);
  al_base = static_cast<int64_t>(p.q_full ? q : slice) * p.q_stride + static_cast<int64_t>(rs) * p.rs_stride +
            static_cast<int64_t>(cs) * p.cs_stride;
  int S[kMaxOrder];
  std_base = 0;
  if (!fill_sectors(p.g, p.row, rs, q, S, p.chg) || !fill_sectors(p.g, p.col, cs, q, S, p.chg)) return false;
  int64_t sb = 0;
  for (int m = 0; m < p.order - 1; ++m) sb = sb * p.hs[m] + S[m];
  std_base = sb * p.blk_elems;
  return true;
}
__host__ __device__ inline bool block_bases(const XformParams& p, int64_t blk, int64_t& std_base,
                                            int64_t& al_base) {
  if (p.nblocks <= INT32_MAX) return block_bases_t<int32_t>(p, static_cast<int32_t>(blk), std_base, al_base);
  return block_bases_t<int64_t>(p, blk, std_base, al_base);
}

// Source and destination offsets of batch row `row` (mixed radix over the batch
// dims, the last one fastest), added to so / dof.
template <typename I>
__host__ __device__ inline void batch_offsets(const XformParams& p, I row, int64_t& so, int64_t& dof) {
  for (int i = p.nbatch - 1; i >= 0; --i) {
    const I b = static_cast<I>(p.bsize[i]);
    const I qd = row / b;
    const I d = row - qd * b;
    row = qd;
    so += static_cast<int64_t>(d) * p.bss[i];
    dof += static_cast<int64_t>(d) * p.bds[i];
  }
}

// Entry i of an offset table for auxiliary sector q: the group's stored sectors
// are the digits of i / n_inner, its in-block indices those of i % n_inner
// (row-major in group order); the implicit sector solves the group's delta.
// (32-bit division where the entry index fits: the tables of large groups have
// millions of entries, and 64-bit division is many times slower on the device)
template <typename I>
__host__ __device__ inline int64_t group_offset_t(const OffsetParams& p, int q, I i) {
  const I n_inner = static_cast<I>(p.n_inner);
  const I digits = i / n_inner;
  I inner = i - digits * n_inner;
  int S[kMaxOrder];
  (void)fill_sectors(p.g, p.grp, digits, q, S, p.chg);   // offset tables: no subgroup modes
  int64_t off = 0;
  for (int j = p.grp.count - 1; j >= 0; --j) {
    const I dim = static_cast<I>(p.dim[j]);
    const I d = inner % dim;
    inner /= dim;
    off += static_cast<int64_t>(d) * p.stride[j] + static_cast<int64_t>(S[p.grp.pos[j]]) * p.weight[j];
  }
  return off;
}
__host__ __device__ inline int64_t group_offset(const OffsetParams& p, int q, int64_t i) {
  if (p.count <= INT32_MAX) return group_offset_t<int32_t>(p, q, static_cast<int32_t>(i));
  return group_offset_t<int64_t>(p, q, i);
}

// Entry i of an offset table for auxiliary sector q, in reals: complex
// operands double every offset, and their column tables hold (re, im) of each
// column at 2c, 2c + 1.
__host__ __device__ inline int64_t table_entry(const OffsetParams& p, int q, int64_t i) {
  if (p.affine) return q * p.aff_q + i * p.aff_i;
  int comp = 0;
  if (p.pairs) {
    comp = static_cast<int>(i & 1);
    i >>= 1;
  }
  return p.scale * group_offset(p, q, i) + comp;
}

}  // namespace symt

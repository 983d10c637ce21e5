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
// `digits` (base |G|, first most significant); the last one solves the
// group's delta.  The deltas hold on charges: with charge tables `chg`
// ([mode][label -> charge | charge -> label][|G|], nullptr for identity) the
// stored labels are mapped to charges and the solved charge back to a label.
__host__ __device__ inline void fill_sectors(const GroupDesc& g, const SectorGroup& sg,
                                             int64_t digits, int q, int* S, const int32_t* chg) {
  if (sg.count == 0) return;        // an empty group only pins Q
  int acc = 0;
  for (int i = sg.count - 2; i >= 0; --i) {
    const int d = static_cast<int>(digits % g.size);
    digits /= g.size;
    S[sg.pos[i]] = d;
    const int c = chg ? chg[(2 * sg.pos[i]) * g.size + d] : d;
    acc = dg_add(g, acc, dg_times(g, sg.coef[i], c));
  }
  const int rhs = dg_add(g, dg_times(g, sg.alpha, q), sg.beta);
  const int last = sg.pos[sg.count - 1];
  const int c = dg_times(g, sg.coef[sg.count - 1], dg_add(g, rhs, dg_neg(g, acc)));
  S[last] = chg ? chg[(2 * last + 1) * g.size + c] : c;
}

// Aligned block index -> (standard-form element offset, aligned element offset).
__host__ __device__ inline void block_bases(const XformParams& p, int64_t blk, int64_t& std_base,
                                            int64_t& al_base) {
  const int64_t cs = blk % p.gpow_col;
  const int64_t t = blk / p.gpow_col;
  const int64_t rs = t % p.gpow_row;
  const int q = p.q_pin >= 0 ? p.q_pin : static_cast<int>(t / p.gpow_row);
  int S[kMaxOrder];
  fill_sectors(p.g, p.row, rs, q, S, p.chg);
  fill_sectors(p.g, p.col, cs, q, S, p.chg);
  int64_t sb = 0;
  for (int m = 0; m < p.order - 1; ++m) sb = sb * p.g.size + S[m];
  std_base = sb * p.blk_elems;
  al_base = q * p.q_stride + rs * p.rs_stride + cs * p.cs_stride;
}

// Entry i of an offset table for auxiliary sector q: the group's stored sectors
// are the digits of i / n_inner, its in-block indices those of i % n_inner
// (row-major in group order); the implicit sector solves the group's delta.
__host__ __device__ inline int64_t group_offset(const OffsetParams& p, int q, int64_t i) {
  int64_t digits = i / p.n_inner;
  int64_t inner = i - digits * p.n_inner;
  int S[kMaxOrder];
  fill_sectors(p.g, p.grp, digits, q, S, p.chg);
  int64_t off = 0;
  for (int j = p.grp.count - 1; j >= 0; --j) {
    const int64_t d = inner % p.dim[j];
    inner /= p.dim[j];
    off += d * p.stride[j] + static_cast<int64_t>(S[p.grp.pos[j]]) * p.weight[j];
  }
  return off;
}

}  // namespace symt

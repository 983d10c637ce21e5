// Host replay of the library's index arithmetic: no GPU, built with g++ and
// AddressSanitizer + UndefinedBehaviorSanitizer by tests/test_host_replay.py.
//
// It plans random contractions with the library's own planner (plan.cpp) and,
// with the index functions the kernels share (xform_index.hpp, sk_index.hpp),
// walks every loop of the launches the library would make, checking:
//  * transforms (copy and tiled-transpose modes, every precision, whole forms
//    and workspace slices): every read and write in bounds, vector accesses
//    aligned and inside their run, every destination element written exactly
//    once and every live source element read exactly once (a bijection);
//  * offset tables of the fused product: U, V and W tables map (Q, row, col)
//    one-to-one onto the stored elements, and the register tiles' load
//    addresses (row offset + one column offset per K-step) equal the table
//    offsets of every element they load, for every K-step layout the planner
//    allows (plain steps, steps run by run, K-major A, V in place);
//  * stream-K: every (tile, K-iteration) is multiplied exactly once, pieces
//    land inside the buffer, each piece slot is written once, and the fixup
//    sums exactly the pieces of its tile in increasing K order; split K covers
//    each tile's K-steps once with partial tiles inside the buffer.
// Exit status 0 when every check passes; the first failures are printed.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "plan.hpp"
#include "sk_index.hpp"
#include "symtensor.h"
#include "xform_index.hpp"

using namespace symt;

namespace {

int g_failures = 0;
int64_t g_checks = 0;
int64_t g_bf16_il = 0;     // transforms writing split-bf16 planes interleaved by K-steps
int64_t g_bf16_fa = 0;     // split-bf16 plans whose wide tile reads binary32 U in place
std::string g_case;

void fail(const char* what, long long a = 0, long long b = 0) {
  if (++g_failures <= 20) std::fprintf(stderr, "FAIL [%s]: %s (%lld, %lld)\n", g_case.c_str(), what, a, b);
}
#define CHECK(cond, what, a, b) \
  do {                          \
    ++g_checks;                 \
    if (!(cond)) fail(what, (long long)(a), (long long)(b)); \
  } while (0)

struct Rng {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  int below(int n) { return static_cast<int>(next() % static_cast<uint64_t>(n)); }
  bool coin() { return next() & 1; }
};

// One operand descriptor with the storage it points to.
struct Desc {
  std::string signs;
  int32_t charge = 0;
  std::vector<int64_t> dims;
  std::vector<int32_t> tables;   // empty: identity
  std::vector<int32_t> sectors;  // empty: |G| each
  int32_t dtype = SYMT_F64;
  symt_tensor t{};
  void bind() {
    t.nmodes = static_cast<int32_t>(signs.size());
    t.signs = signs.c_str();
    t.charge = charge;
    t.dims = dims.data();
    t.dtype = dtype;
    t.data = nullptr;
    t.mode_charges = tables.empty() ? nullptr : tables.data();
    t.sectors = sectors.empty() ? nullptr : sectors.data();
  }
};

struct Case {
  std::string einsum;
  symt_group g{};
  Desc u, v, w;
  int32_t compute = 0;
};

int group_size(const symt_group& g) {
  int n = 1;
  for (int f = 0; f < g.nfactors; ++f) n *= g.order[f];
  return n;
}

// ---------------------------------------------------------------------------
// Transforms
// ---------------------------------------------------------------------------
// Walks every access of one transform launch (k_xform_copy / k_xform_transpose):
// src_n / dst_n are the elements of the source and destination (per plane for
// a split destination).  Counts land in `written` (2 dst_n with planes) and `read`.
void replay_xform(const XformParams& x, int64_t src_n, int64_t dst_n, bool dst_split, std::vector<uint8_t>& written,
                  std::vector<uint8_t>& read) {
  const int64_t nwg = x.nblocks * x.tiles_per_block;
  auto write = [&](int64_t d) {
    CHECK(d >= 0 && d < dst_n, "destination out of bounds", d, dst_n);
    if (d < 0 || d >= dst_n) return;
    if (dst_split && x.il) {
      // planes interleaved by 32-deep K-steps: hi at 2 d - d % 32, lo 32 after
      const int64_t h = 2 * d - (d & 31), e = h + x.plane;
      CHECK(x.plane == 32, "interleaved hi-to-lo distance", x.plane, 32);
      CHECK(h >= 0 && e < 2 * dst_n, "interleaved plane element out of bounds", e, 2 * dst_n);
      if (h < 0 || e >= 2 * dst_n) return;
      CHECK(written[h] == 0 && written[e] == 0, "interleaved plane element written twice", h, 0);
      written[h]++;
      written[e]++;
      return;
    }
    CHECK(written[d] == 0, "destination written twice", d, 0);
    written[d]++;
    if (dst_split) {
      const int64_t e = d + x.plane;
      CHECK(e >= dst_n && e < 2 * dst_n, "lo plane out of bounds", e, dst_n);
      if (e >= 0 && e < 2 * dst_n) written[e]++;
    }
  };
  auto readsrc = [&](int64_t s) {
    CHECK(s >= 0 && s < src_n, "source out of bounds", s, src_n);
    if (s >= 0 && s < src_n) {
      CHECK(read[s] == 0, "source element read twice", s, 0);
      read[s]++;
    }
  };
  for (int64_t wg = 0; wg < nwg; ++wg) {
    const int64_t blk = wg / x.tiles_per_block;
    int64_t sb = 0, ab = 0;
    const bool live = block_bases(x, blk, sb, ab);
    if (!live && !x.to_aligned) continue;
    const int64_t src_base = x.to_aligned ? sb : ab;
    const int64_t dst_base = x.to_aligned ? ab : sb;
    if (x.mode == 0) {
      const int64_t tile = wg - blk * x.tiles_per_block;
      const int64_t row_tile = tile / x.run_tiles;
      const int64_t c_begin = (tile - row_tile * x.run_tiles) * x.run_chunk;
      const int64_t c_end = std::min(c_begin + x.run_chunk, x.run_len);
      const int64_t r0 = row_tile * x.rows_per_tile;
      const int nr = static_cast<int>(std::min<int64_t>(x.rows - r0, x.rows_per_tile));
      // (the kernel moves them 1024 at a time through its LDS row table)
      CHECK(nr >= 1, "copy tile without rows", nr, x.rows);
      const int V = x.vec;
      CHECK(c_begin % V == 0, "vector chunk start", c_begin, V);
      for (int r = 0; r < nr; ++r) {
        int64_t rem = r0 + r, so = 0, dof = 0;
        for (int i = x.nbatch - 1; i >= 0; --i) {
          const int64_t qd = rem / x.bsize[i];
          const int64_t d = rem - qd * x.bsize[i];
          rem = qd;
          so += d * x.bss[i];
          dof += d * x.bds[i];
        }
        const int64_t s0 = src_base + so, d0 = dst_base + dof;
        for (int64_t c = c_begin; c < c_end; c += V) {
          if (V > 1) {
            CHECK(c + V <= c_end, "vector past its run", c, c_end);
            CHECK((s0 + c) % V == 0 && (d0 + c) % V == 0, "vector access misaligned", s0 + c, d0 + c);
            CHECK(x.run_ss == 1 && x.run_ds == 1, "vector along a strided run", x.run_ss, x.run_ds);
          }
          for (int j = 0; j < V; ++j) {
            if (live) readsrc(s0 + (c + j) * x.run_ss);
            write(d0 + (c + j) * x.run_ds);
          }
        }
      }
    } else {
      int64_t rem = wg - blk * x.tiles_per_block;
      const int64_t tb = rem % x.tiles_t;
      rem /= x.tiles_t;
      const int64_t ta = rem % x.tiles_run;
      int64_t row = rem / x.tiles_run;
      int64_t so = src_base, dof = dst_base;
      for (int i = x.nbatch - 1; i >= 0; --i) {
        const int64_t qd = row / x.bsize[i];
        const int64_t d = row - qd * x.bsize[i];
        row = qd;
        so += d * x.bss[i];
        dof += d * x.bds[i];
      }
      const int64_t a0 = ta * 64, b0 = tb * 64;
      const int na = static_cast<int>(std::min<int64_t>(x.run_len - a0, 64));
      const int nb = static_cast<int>(std::min<int64_t>(x.t_len - b0, 64));
      auto offs = [](int64_t i, int n, const int64_t* size, const int64_t* ss, const int64_t* ds, int64_t& s,
                     int64_t& d) {
        s = 0;
        d = 0;
        for (int k = 0; k < n; ++k) {
          const int64_t q = i / size[k];
          const int64_t c = i - q * size[k];
          i = q;
          s += c * ss[k];
          d += c * ds[k];
        }
      };
      if (x.tr_write) {
        // the kernel ranks the A elements by destination offset: a permutation
        std::vector<int64_t> adst(static_cast<size_t>(na));
        for (int ia = 0; ia < na; ++ia) {
          int64_t as;
          offs(a0 + ia, x.na, x.asize, x.ass, x.ads, as, adst[ia]);
        }
        std::vector<int> seen(static_cast<size_t>(na), 0);
        for (int t = 0; t < na; ++t) {
          int rk = 0;
          for (int u = 0; u < na; ++u) rk += adst[u] < adst[t] || (adst[u] == adst[t] && u < t);
          CHECK(rk >= 0 && rk < na, "transpose write rank out of range", rk, na);
          if (rk >= 0 && rk < na) seen[rk]++;
        }
        for (int r = 0; r < na; ++r) CHECK(seen[r] == 1, "transpose write ranks not a permutation", r, seen[r]);
      }
      for (int ia = 0; ia < na; ++ia) {
        int64_t as, ad;
        offs(a0 + ia, x.na, x.asize, x.ass, x.ads, as, ad);
        for (int ib = 0; ib < nb; ++ib) {
          int64_t bs, bd;
          offs(b0 + ib, x.nb, x.tsize, x.tss, x.tds, bs, bd);
          if (live) readsrc(so + as + bs);
          write(dof + ad + bd);
        }
      }
    }
  }
}

// Aligned matrix of operand 0/1/2 in reals: rows and columns per Q slice.
void aligned_dims(const Plan& p, int op, int64_t& rows, int64_t& cols) {
  const int64_t rm = p.cplx && op == 1 ? 2 : 1;   // complex V: two real rows per complex row
  if (op == 0) { rows = p.M; cols = p.gk; }
  else if (op == 1) { rows = p.Kd * rm; cols = p.gn; }
  else { rows = p.M; cols = p.gn; }
}

// k_cplx_rows over a complex V_al of `nsl` slices: row 2r + 1 from row 2r.
// Outside [lo, hi) (slices a standalone transform cleared instead of moving)
// it rewrites zeros: only its bounds are checked there.
// Split-bf16 planes (planes: true) store the real V K fastest at pitch kp:
// k_cplx_rows_planes fills (2k + 1, 2n) and (2k + 1, 2n + 1) of both planes.
void replay_cplx_rows_planes(const Plan& p, int64_t nsl, int64_t al_n, int64_t kp, std::vector<uint8_t>& written,
                             int64_t lo, int64_t hi) {
  const int64_t pairs = p.N;
  for (int64_t i = 0; i < nsl * pairs * p.Kd; ++i) {
    const int64_t k = i % p.Kd, t = i / p.Kd, n = t % pairs, sl = t / pairs;
    const int64_t re = (sl * 2 * pairs + 2 * n) * kp + 2 * k, im = re + kp;
    CHECK(re >= 0 && im + 1 < al_n, "complex plane row out of bounds", im + 1, al_n);
    if (re < 0 || im + 1 >= al_n || re < lo || re >= hi) continue;
    CHECK(written[re] == 1 && written[im] == 1, "complex plane row from an unwritten even row", re, 0);
    for (int64_t e : {re + 1, im + 1})
      for (int64_t pl = 0; pl < 2; ++pl) {
        CHECK(written[e + pl * al_n] == 0, "complex plane row written twice", e, pl);
        written[e + pl * al_n]++;
      }
  }
}

void replay_cplx_rows(const Plan& p, int64_t nsl, int64_t al_n, std::vector<uint8_t>& written, int64_t lo,
                      int64_t hi) {
  const int64_t pairs = p.N;
  for (int64_t i = 0; i < nsl * p.Kd * pairs; ++i) {
    const int64_t c = i % pairs, r = i / pairs;
    const int64_t even = (2 * r) * (2 * pairs) + 2 * c;
    CHECK(even >= 0 && even + 2 * pairs + 1 < al_n, "complex odd row out of bounds", even, al_n);
    if (even < 0 || even + 2 * pairs + 1 >= al_n) continue;
    if (even < lo || even >= hi) continue;
    CHECK(written[even] == 1 && written[even + 1] == 1, "complex odd row from an unwritten even row", even, 0);
    for (int64_t e : {even + 2 * pairs, even + 2 * pairs + 1}) {
      CHECK(written[e] == 0, "complex odd row written twice", e, 0);
      written[e]++;
    }
  }
}

void check_transforms(const Plan& p) {
  const int G = p.g.size;
  const int kind = p.compute == SYMT_COMPUTE_F64 ? 0 : p.compute == SYMT_COMPUTE_F32 ? 1 : 2;
  const int al_bytes = kind == 0 ? 8 : kind == 1 ? 4 : 2;
  for (int op = 0; op < 3; ++op) {
    const OperandDesc& X = op == 0 ? p.U : op == 1 ? p.V : p.W;
    if (X.elems == 0) continue;
    const int64_t reals = X.elems * (p.cplx ? 2 : 1);
    int64_t rows, cols;
    aligned_dims(p, op, rows, cols);
    const int64_t per_slice = rows * cols;
    for (int slice_only = 0; slice_only < 2; ++slice_only) {
      // standalone transforms take identity tables only (their aligned layouts are by label)
      if (!slice_only && p.charges) continue;
      const bool to_al = op != 2;
      const bool split = to_al && kind == 2;
      const int in_bytes = to_al ? real_bytes(X.dtype) : (p.compute == SYMT_COMPUTE_F32 ? 4 : 8);
      const int out_bytes = to_al ? al_bytes : real_bytes(X.dtype);
      const XformParams x0 = make_xform(p, op, to_al, in_bytes, out_bytes, split, slice_only != 0);
      for (int scalar = 0; scalar < 2; ++scalar) {
        XformParams x = x0;
        if (scalar) {
          if (x.vec == 1) continue;
          x.vec = 1;     // operands that are not 16-byte aligned
        }
        const int64_t nsl = slice_only ? p.nq : G;
        // the contraction's split-bf16 planes hold K at pitch kpad (pad unwritten)
        const bool kpad = slice_only && kind == 2 && op < 2 && p.kpad != p.gk;
        const int64_t slice_n = kpad ? (op == 0 ? p.M * p.kpad : p.kpad * p.gn) : per_slice;
        const int64_t al_n = nsl * slice_n;
        CHECK(x.plane == al_n || !split || x.il, "hi-to-lo plane distance", x.plane, al_n);
        // interleaved planes: the contraction's own aligned operands, K a whole number of K-steps
        CHECK(!x.il || (split && slice_only && op < 2 && p.bf16_il && !p.cplx && p.kpad % 32 == 0),
              "interleaved planes outside the wide split-bf16 product", op, p.kpad);
        if (x.il && !scalar) ++g_bf16_il;
        if (to_al) {
          std::vector<uint8_t> written(static_cast<size_t>(al_n) * (split ? 2 : 1), 0);
          std::vector<uint8_t> read(static_cast<size_t>(reals), 0);
          replay_xform(x, reals, al_n, split, written, read);
          // every element of the moved slices written once (dead aligned blocks as
          // zeros); with Q pinned the standalone transform moves one slice (the
          // others are cleared by a separate launch)
          int64_t lo = 0, hi = al_n;
          if (!slice_only && pinned_form(p, op)) {
            lo = static_cast<int64_t>(p.q_pin) * per_slice;
            hi = lo + per_slice;
          }
          if (p.cplx && op == 1) {
            if (kind == 2)
              replay_cplx_rows_planes(p, nsl, al_n, kpad ? p.kpad : p.gk, written, lo, hi);
            else
              replay_cplx_rows(p, nsl, al_n, written, lo, hi);
          }
          for (int64_t d = 0; d < al_n; ++d) {
            const uint8_t want = d >= lo && d < hi && !(kpad && d % p.kpad >= p.gk) ? 1 : 0;
            const int64_t h = x.il ? 2 * d - (d & 31) : d, e = x.il ? h + 32 : d + al_n;
            CHECK(written[h] == want, "aligned element not written exactly once", d, written[h]);
            if (split) CHECK(written[e] == want, "lo plane element not written exactly once", d, written[e]);
          }
        } else {
          std::vector<uint8_t> written(static_cast<size_t>(reals), 0);
          std::vector<uint8_t> read(static_cast<size_t>(al_n), 0);
          replay_xform(x, al_n, reals, false, written, read);
          // with every Q slice live and no subgroup mode, W is covered exactly
          if (p.nq == G && !p.subgroups)
            for (int64_t d = 0; d < reals; ++d) CHECK(written[d] == 1, "W element not written exactly once", d, written[d]);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Offset tables and the fused product's load addresses
// ---------------------------------------------------------------------------
std::vector<int64_t> table(const OffsetParams& o, int G) {
  std::vector<int64_t> t(static_cast<size_t>(G * o.count));
  for (int q = 0; q < G; ++q)
    for (int64_t i = 0; i < o.count; ++i) t[q * o.count + i] = table_entry(o, q, i);
  return t;
}

void check_bijection(const std::vector<int64_t>& R, const std::vector<int64_t>& C, int G, int64_t rows,
                     int64_t cols, int64_t reals, const char* what) {
  std::vector<uint8_t> hit(static_cast<size_t>(reals), 0);
  for (int q = 0; q < G; ++q)
    for (int64_t r = 0; r < rows; ++r)
      for (int64_t c = 0; c < cols; ++c) {
        const int64_t off = R[q * rows + r] + C[q * cols + c];
        CHECK(off >= 0 && off < reals, what, off, reals);
        if (off >= 0 && off < reals) hit[off]++;
      }
  for (int64_t e = 0; e < reals; ++e) CHECK(hit[e] == 1, what, e, hit[e]);
}

// The row-streaming product (K and N at most 64): the index walk of one launch
// over tables (empty vector: the aligned row-major form).  Every A and B read
// inside its operand, every C element written exactly once.
// (`resident`: workgroups the device holds at once; the launcher asks the
// runtime, the replay tries several)
void replay_rows(int64_t resident, int64_t batch, int64_t M, int64_t N, int64_t K, const std::vector<int64_t>& ra,
                 const std::vector<int64_t>& ca, const std::vector<int64_t>& rb, const std::vector<int64_t>& cb,
                 const std::vector<int64_t>& rc, const std::vector<int64_t>& cc, int64_t a_n, int64_t b_n,
                 int64_t c_n, int row_groups, bool trans, int rv = 1, int kv = 1, int ko = 1) {
  // (rv > 1: lane r of a 16 rv-row group loads rows rv r .. rv r + rv - 1 of one K
  // index with one vector load; MFMA output row p of vector element t is row rv p + t)
  const int waves = 4, rows = 16 * row_groups * rv;
  const int64_t ks = (K + 3) / 4, tn = (N + 15) / 16;
  const int64_t blocks = (M + rows - 1) / rows;
  const int64_t want = std::max<int64_t>(1, resident / std::max<int64_t>(batch, 1));
  const int64_t gx = std::min<int64_t>((blocks + waves - 1) / waves, want);
  std::vector<uint8_t> written(static_cast<size_t>(c_n), 0);
  for (int64_t q = 0; q < batch; ++q) {
    for (int64_t k = 0; k < 4 * ks; ++k)
      for (int64_t n = 0; n < 16 * tn; ++n) {
        if (k >= K || n >= N) continue;
        const int64_t b = rb.empty() ? (q * K + k) * N + n : rb[q * K + k] + cb[q * N + n];
        CHECK(b >= 0 && b < b_n, "row product B read out of bounds", b, b_n);
      }
    for (int64_t x = 0; x < gx; ++x)
      for (int w = 0; w < waves; ++w)
        for (int64_t blk = x * waves + w; blk < blocks; blk += gx * waves) {
          const int64_t m0 = blk * rows;
          for (int lane = 0; lane < 64; ++lane) {
            for (int g = 0; g < row_groups * rv; ++g) {
              const int i = g / rv, t = g % rv;
              const int64_t m = std::min<int64_t>(m0 + i * 16 * rv + rv * (lane & 15), M - rv);
              const int64_t rbase = ra.empty() ? (q * M + m) * K : ra[q * M + m];
              if (rv > 1 && t == 0) {
                CHECK(M % rv == 0 && rbase % rv == 0, "row vector of A misaligned", m, rbase);
                for (int u = 1; u < rv; ++u)
                  CHECK(ra[q * M + m + u] == rbase + u, "row vector of A not contiguous", m, u);
              }
              for (int64_t st = 0; st < ks && t == 0; ++st) {
                // (kv > 1: one vector of kv K indices per group of kv steps)
                // (ko > 1: binary32's K order, 4 ko (st / ko) + ko kq + st % ko)
                if (kv > 1 && st % kv != 0) continue;
                const int64_t k = ko > 1 ? 4 * ko * (st / ko) + ko * (lane >> 4) + st % ko : 4 * st + (lane >> 4);
                if (k >= K) continue;
                const int64_t a = rbase + (ca.empty() ? k : ca[q * K + k]);
                CHECK(a >= 0 && a + rv * kv <= a_n, "row product A read out of bounds", a, a_n);
                CHECK(a % (rv * kv) == 0, "vector load of A misaligned", a, rv * kv);
                for (int j = 1; j < kv && !ca.empty(); ++j)
                  CHECK(ca[q * K + k + j] == ca[q * K + k] + j, "K vector of A not contiguous", k, j);
              }
              // stores: both accumulator row layouts cover rows m0 + 16 i + 0..15
              // (trans: the lane's row is lane % 16, its columns those rows; rv > 1:
              // MFMA output row p of vector element t is row rv p + t)
              for (int r = 0; r < 4; ++r) {
                const int64_t acc_row = (lane >> 4) + 4 * r;
                const int64_t row = m0 + i * 16 * rv + (trans ? (lane & 15) : rv * acc_row + t);
                if (row >= M) continue;
                const int64_t crow = rc.empty() ? (q * M + row) * N : rc[q * M + row];
                for (int64_t j = 0; j < tn; ++j) {
                  const int64_t col = j * 16 + (trans ? acc_row : (lane & 15));
                  if (col >= N) continue;
                  const int64_t c = crow + (cc.empty() ? col : cc[q * N + col]);
                  CHECK(c >= 0 && c < c_n, "row product C write out of bounds", c, c_n);
                  if (c >= 0 && c < c_n) {
                    CHECK(written[c] == 0, "row product C written twice", c, 0);
                    written[c]++;
                  }
                }
              }
            }
          }
        }
  }
  int64_t total = 0;
  for (uint8_t v : written) total += v;
  CHECK(total == batch * M * N, "row product C elements not all written", total, batch * M * N);
}

// The long-K product (M and N at most 64): the index walk of its two launches.
// Every K index multiplied exactly once per slice, every A and B read inside its
// operand, partials inside their buffer, every C element written exactly once.
void replay_tallk(int64_t batch, int64_t M, int64_t N, int64_t K, const std::vector<int64_t>& ra,
                  const std::vector<int64_t>& ca, const std::vector<int64_t>& rb, const std::vector<int64_t>& cb,
                  const std::vector<int64_t>& rc, const std::vector<int64_t>& cc, int64_t a_n, int64_t b_n,
                  int64_t c_n) {
  const int ranges = tallk_ranges(batch, K);
  const int kc = tallk_range(K, ranges);
  CHECK(kc % 16 == 0 && static_cast<int64_t>(kc) * ranges >= K, "long-K ranges do not cover K", kc, ranges);
  const int64_t part_n = batch * ranges * M * N;
  std::vector<uint8_t> written(static_cast<size_t>(c_n), 0);
  std::vector<uint8_t> part_w(static_cast<size_t>(part_n), 0);
  const int64_t tm = (M + 15) / 16, tn = (N + 15) / 16;
  for (int64_t q = 0; q < batch; ++q) {
    std::vector<uint8_t> cover(static_cast<size_t>(K), 0);
    for (int x = 0; x < ranges; ++x) {
      const int64_t k_begin = static_cast<int64_t>(x) * kc, k_end = std::min<int64_t>(K, k_begin + kc);
      for (int w = 0; w < 4; ++w)
        for (int64_t g = k_begin + w * 16; g < k_end; g += 64)
          for (int lane = 0; lane < 64; ++lane)
            for (int u = 0; u < 4; ++u) {
              const int64_t k = g + 4 * u + (lane >> 4);
              if (k >= k_end) continue;
              if ((lane & 15) == 0) cover[k]++;   // one lane per K index and row tile
              const int64_t ak = ca.empty() ? k : ca[q * K + k];
              const int64_t bk = rb.empty() ? (q * K + k) * N : rb[q * K + k];
              for (int64_t i = 0; i < tm; ++i) {
                const int64_t m = 16 * i + (lane & 15);
                if (m >= M) continue;
                const int64_t a = (ra.empty() ? (q * M + m) * K : ra[q * M + m]) + ak;
                CHECK(a >= 0 && a < a_n, "long-K A read out of bounds", a, a_n);
              }
              // A along K (rows (lane / 16) + 4 j, K index g + lane % 16), once per group
              if (u == 0) {
                const int64_t kk = g + (lane & 15);
                if (kk < k_end)
                  for (int64_t j = 0; j < 4 * tm; ++j) {
                    const int64_t m = (lane >> 4) + 4 * j;
                    if (m >= M) continue;
                    const int64_t a = (ra.empty() ? (q * M + m) * K : ra[q * M + m]) + (ca.empty() ? kk : ca[q * K + kk]);
                    CHECK(a >= 0 && a < a_n, "long-K A read along K out of bounds", a, a_n);
                    CHECK(m < 16 * tm, "long-K slab row past the tile", m, 16 * tm);
                  }
              }
              for (int64_t j = 0; j < tn; ++j) {
                const int64_t n = 16 * j + (lane & 15);
                if (n >= N) continue;
                const int64_t b = bk + (cb.empty() ? n : cb[q * N + n]);
                CHECK(b >= 0 && b < b_n, "long-K B read out of bounds", b, b_n);
              }
            }
      for (int64_t e = 0; e < M * N; ++e) {
        const int64_t pe = (q * ranges + x) * M * N + e;
        CHECK(pe >= 0 && pe < part_n && part_w[pe] == 0, "long-K partial out of bounds or twice", pe, part_n);
        if (pe >= 0 && pe < part_n) part_w[pe]++;
      }
    }
    for (int64_t k = 0; k < K; ++k) CHECK(cover[k] == 1, "long-K index not multiplied once", k, cover[k]);
    for (int64_t e = 0; e < M * N; ++e) {
      const int64_t m = e / N, n = e % N;
      const int64_t c = rc.empty() ? (q * M + m) * N + n : rc[q * M + m] + cc[q * N + n];
      CHECK(c >= 0 && c < c_n, "long-K C write out of bounds", c, c_n);
      if (c >= 0 && c < c_n) {
        CHECK(written[c] == 0, "long-K C written twice", c, 0);
        written[c]++;
      }
    }
  }
}

// The long-K product's global-to-LDS variant (taken where tallk_groups holds):
// each wave's 16-deep groups of K through its LDS ring.  Checks that every group of
// K lies in one contiguous run of A's rows and one affine run of B's rows, that
// B's 16-byte column chunks are contiguous, every load is 16-byte aligned and
// inside its operand, every K index is multiplied once, and that the swizzled
// LDS slots hand each MFMA operand read the element it stands for.
int tk_bswz_host(int elem, int np, int k) {
  const int row_bytes = np * elem;
  if (elem == 8) return row_bytes % 256 == 0 ? (k & 1) << 3 : 0;
  if (row_bytes % 256 == 0) return (k & 3) << 2;
  if (row_bytes % 256 == 128) return ((k >> 1) & 1) << 2;
  return 0;
}

int64_t g_tallk_dma = 0;   // plans whose long-K product takes the global-to-LDS variant
int64_t g_at_dma = 0;      // plans whose product can read K-major A on global-to-LDS tiles
int64_t g_row_vec = 0;     // plans whose row-streaming product loads row vectors of K-major A
int64_t g_a_kvec = 0;      // plans whose register tiles load K vectors of K-major A
int64_t g_k_vec = 0;       // plans whose row-streaming product loads K vectors of A

void replay_tallk_dma(int elem, int64_t batch, int64_t M, int64_t N, int64_t K, const std::vector<int64_t>& ra,
                      const std::vector<int64_t>& ca, const std::vector<int64_t>& rb, const std::vector<int64_t>& cb,
                      int64_t ldb, int64_t a_n, int64_t b_n) {
  const int VE = 16 / elem, GK = 16, CPR = GK / VE;
  auto aswz = [&](int r) { return elem == 8 ? (r >> 1) & 7 : (r >> 2) & 3; };
  if (K % GK != 0 || N % VE != 0) return;   // the launcher keeps the register variant
  ++g_tallk_dma;
  const int tm = static_cast<int>((M + 15) / 16), tn = static_cast<int>((N + 15) / 16);
  const int MP = 16 * tm, NP = 16 * tn, BCH = NP / VE;
  const int ranges = tallk_ranges(batch, K);
  const int kc = tallk_range(K, ranges);
  for (int64_t q = 0; q < batch; ++q) {
    std::vector<uint8_t> cover(static_cast<size_t>(K), 0);
    for (int x = 0; x < ranges; ++x) {
      const int64_t k_begin = static_cast<int64_t>(x) * kc, k_end = std::min<int64_t>(K, k_begin + kc);
      for (int w = 0; w < 4; ++w)
        for (int64_t g = k_begin + w * GK; g < k_end; g += 4 * GK) {
          CHECK(g + GK <= k_end, "long-K group past its range", g, k_end);
          const int64_t acol = ca.empty() ? g : ca[q * K + g];
          const int64_t brow = rb.empty() ? (q * K + g) * N : rb[q * K + g];
          for (int j = 0; j < GK; ++j) {
            cover[g + j]++;
            if (!ca.empty()) CHECK(ca[q * K + g + j] == acol + j, "long-K A group not contiguous", g, j);
            if (!rb.empty()) CHECK(rb[q * K + g + j] == brow + j * ldb, "long-K B group not affine", g, j);
          }
          // LDS labels: A slot (r, pos) holds row min(r, M - 1), K chunk pos ^ aswz(r)
          std::vector<int64_t> lab_a(static_cast<size_t>(MP) * GK), lab_b(static_cast<size_t>(GK) * NP);
          for (int slot = 0; slot < MP * CPR; ++slot) {
            const int r = slot / CPR, c = (slot % CPR) ^ aswz(r);
            CHECK(c >= 0 && c < CPR, "long-K A swizzle past the row", c, CPR);
            const int64_t gr = std::min<int64_t>(r, M - 1);
            const int64_t a = (ra.empty() ? (q * M + gr) * K : ra[q * M + gr]) + c * VE + acol;
            CHECK(a % VE == 0 && a >= 0 && a + VE <= a_n, "long-K A chunk misaligned or out of bounds", a, a_n);
            for (int e = 0; e < VE; ++e) lab_a[slot * VE + e] = gr * GK + c * VE + e;
          }
          for (int slot = 0; slot < GK * BCH; ++slot) {
            const int k = slot / BCH, c = (slot % BCH) ^ tk_bswz_host(elem, NP, k);
            CHECK(c >= 0 && c < BCH, "long-K B swizzle past the row", c, BCH);
            const int64_t gn = std::min<int64_t>(static_cast<int64_t>(c) * VE, N - VE);
            if (!cb.empty())
              for (int e = 1; e < VE; ++e)
                CHECK(cb[q * N + gn + e] == cb[q * N + gn] + e, "long-K B chunk not contiguous", gn, e);
            const int64_t b = brow + k * ldb + (cb.empty() ? gn : cb[q * N + gn]);
            CHECK(b % VE == 0 && b >= 0 && b + VE <= b_n, "long-K B chunk misaligned or out of bounds", b, b_n);
            for (int e = 0; e < VE; ++e) lab_b[slot * VE + e] = k * NP + gn + e;
          }
          for (int m = 0; m < M; ++m)
            for (int k = 0; k < GK; ++k) {
              const int idx = m * GK + ((k / VE) ^ aswz(m)) * VE + k % VE;
              CHECK(lab_a[idx] == static_cast<int64_t>(m) * GK + k, "long-K A operand read from the wrong slot", m, k);
            }
          for (int k = 0; k < GK; ++k)
            for (int n = 0; n < N; ++n) {
              const int idx = k * NP + ((n / VE) ^ tk_bswz_host(elem, NP, k)) * VE + n % VE;
              CHECK(lab_b[idx] == static_cast<int64_t>(k) * NP + n, "long-K B operand read from the wrong slot", k, n);
            }
        }
    }
    for (int64_t k = 0; k < K; ++k) CHECK(cover[k] == 1, "long-K group index not multiplied once", k, cover[k]);
  }
}

void check_fused(const Plan& p) {
  if (!(p.fused || p.fused_ua)) return;
  const int G = p.g.size;
  const int cm = p.cplx ? 2 : 1;
  std::vector<int64_t> ra, ca, rc, cc, rb, cb;
  if (p.fused_ua) {
    ra = table(affine_offsets(p, p.M, p.M * p.gk, p.gk), G);
    ca = table(affine_offsets(p, p.gk, 0, 1), G);
    check_bijection(ra, ca, G, p.M, p.gk, G * p.M * p.gk, "U_al affine tables");
  } else {
    ra = table(make_offsets(p, 0, true), G);
    ca = table(make_offsets(p, 0, false), G);
    check_bijection(ra, ca, G, p.M, p.gk, p.U.elems * cm, "U tables not a bijection onto U");
  }
  rc = table(make_offsets(p, 2, true), G);
  cc = table(make_offsets(p, 2, false), G);
  check_bijection(rc, cc, G, p.M, p.gn, p.W.elems * cm, "W tables not a bijection onto W");
  if (p.bf16_wide_fa) {
    // the wide split-bf16 tile reading binary32 U in place: one 16-byte load per
    // run of 4 along K, at ra(Q, m) + ca(Q, k) for k a multiple of 4
    ++g_bf16_fa;
    CHECK(p.fused_ua && p.bf16_il && !p.cplx && p.U.dtype == SYMT_F32 && p.gk % 32 == 0 && p.gk == p.kpad,
          "wide split-bf16 in place outside its conditions", p.gk, p.kpad);
    const std::vector<int64_t> ua = table(make_offsets(p, 0, true), G), uc = table(make_offsets(p, 0, false), G);
    check_bijection(ua, uc, G, p.M, p.gk, p.U.elems, "U tables (wide split-bf16 in place) not a bijection onto U");
    for (int q = 0; q < G; ++q)
      for (int64_t k = 0; k + 3 < p.gk; k += 4) {
        const int64_t c0 = uc[q * p.gk + k];
        for (int i = 1; i < 4; ++i) CHECK(uc[q * p.gk + k + i] == c0 + i, "U's K run of 4 not contiguous", k, i);
        for (int64_t m = 0; m < p.M; ++m) {
          const int64_t off = ua[q * p.M + m] + c0;
          CHECK(off % 4 == 0, "U run of 4 not 16-byte aligned", m, k);
          CHECK(off >= 0 && off + 4 <= p.U.elems, "U run of 4 out of bounds", off, p.U.elems);
        }
      }
  }
  if (!p.cplx && p.w_row_run % 4 == 0) {
    // binary32 tiles store 4 consecutive rows of a column with one 16-byte store
    for (int q = 0; q < G; ++q)
      for (int64_t m = 0; m + 3 < p.M; m += 4) {
        for (int t = 1; t < 4; ++t)
          CHECK(rc[q * p.M + m + t] == rc[q * p.M + m] + t, "W rows not in runs of 4", m, t);
        for (int64_t n = 0; n < p.gn; ++n)
          CHECK((rc[q * p.M + m] + cc[q * p.gn + n]) % 4 == 0, "W run of 4 rows not 16-byte aligned", m, n);
      }
  }
  if (p.fused_b) {
    rb = table(make_offsets(p, 1, true), G);
    cb = table(make_offsets(p, 1, false), G);
    check_bijection(rb, cb, G, p.gk, p.gn, p.V.elems, "V tables not a bijection onto V");
  }
  if (p.compute != SYMT_COMPUTE_BF16X3 && p.M <= 64 && p.gn <= 64) {
    const std::vector<int64_t> none;
    const int64_t b_n = p.fused_b ? p.V.elems : G * p.gk * p.gn;
    replay_tallk(G, p.M, p.gn, p.gk, ra, ca, p.fused_b ? rb : none, p.fused_b ? cb : none, rc, cc,
                 p.fused_ua ? G * p.M * p.gk : p.U.elems * cm, b_n, p.W.elems * cm);
    if (tallk_groups(p))
      replay_tallk_dma(p.compute == SYMT_COMPUTE_F64 ? 8 : 4, G, p.M, p.gn, p.fused_ua ? p.kpad : p.gk, ra, ca,
                       p.fused_b ? rb : none, p.fused_b ? cb : none, p.fused_b ? p.ldb : p.gn,
                       p.fused_ua ? G * p.M * p.kpad : p.U.elems * cm, b_n);
  }
  if (p.compute != SYMT_COMPUTE_BF16X3 && p.gk <= 64 && p.gn <= 64) {
    const std::vector<int64_t> none;
    const int64_t b_n = p.fused_b ? p.V.elems : G * p.gk * p.gn;   // V in place, or V_al
    for (int rg : {1, 2})
      for (int64_t resident : {256, 512, 2048})
        for (bool trans : {false, true})
          replay_rows(resident, G, p.M, p.gn, p.gk, ra, ca, p.fused_b ? rb : none, p.fused_b ? cb : none, rc, cc,
                      p.fused_ua ? G * p.M * p.gk : p.U.elems * cm, b_n, p.W.elems * cm, rg, trans, 1, 1,
                      p.compute == SYMT_COMPUTE_F32 ? 4 : 1);
    // binary32 A with its K index contiguous in aligned runs of 4: K vectors
    const int64_t krun_a = p.fused_ua ? p.gk : p.nK;
    if (p.compute == SYMT_COMPUTE_F32 && !p.a_trans && !p.cplx && krun_a % 4 == 0 && p.gk % 4 == 0) {
      ++g_k_vec;
      for (bool trans : {false, true})
        replay_rows(512, G, p.M, p.gn, p.gk, ra, ca, p.fused_b ? rb : none, p.fused_b ? cb : none, rc, cc,
                    p.fused_ua ? G * p.M * p.gk : p.U.elems * cm, b_n, p.W.elems * cm, 2, trans, 1, 4, 4);
    }
    // binary32 K-major A with 16-byte chunks along M: row vectors of 4 (one row group)
    const int vwr = 4;
    if (p.compute == SYMT_COMPUTE_F32 && p.a_trans && p.a_chunks && p.M % vwr == 0) {
      ++g_row_vec;
      for (int64_t resident : {256, 2048})
        replay_rows(resident, G, p.M, p.gn, p.gk, ra, ca, p.fused_b ? rb : none, p.fused_b ? cb : none, rc, cc,
                    p.U.elems * cm, b_n, p.W.elems * cm, 1, false, vwr, 1, 4);
    }
  }
  if (p.compute == SYMT_COMPUTE_BF16X3) {
    // register tiles split U in registers along 32-deep K-steps of one run
    if (p.fused)
      for (int q = 0; q < G; ++q)
        for (int64_t k = 0; k < p.gk; ++k)
          CHECK(ca[q * p.gk + k] == ca[q * p.gk + (k / 32) * 32] + k % 32, "split-bf16 A step not contiguous", k, q);
    return;
  }
  // Register tiles (BK = 16): K-step kt starts at k0 with kv valid rows.
  const int BK = kFpBK;
  const int spr = p.krun > 0 ? (p.krun + BK - 1) / BK : 0;
  const int64_t nk_all = p.krun > 0 ? p.gk / p.krun * spr : (p.gk + BK - 1) / BK;
  const GemmChoice gc = choose_fp_gemm(G, p.M, p.gn, p.gk, p.compute == SYMT_COMPUTE_F64 ? 8 : 4, true, p.a_trans);
  for (int q = 0; q < G; ++q)
    for (int64_t kt = 0; kt < nk_all; ++kt) {
      int64_t k0, kv;
      if (p.krun > 0) {
        const int64_t run = kt / spr, st = kt - run * spr;
        k0 = run * p.krun + st * BK;
        kv = std::min<int64_t>(BK, p.krun - st * BK);
      } else {
        k0 = kt * BK;
        kv = std::min<int64_t>(BK, p.gk - k0);
      }
      CHECK(k0 + kv <= p.gk, "K-step past K", k0 + kv, p.gk);
      for (int64_t c = 0; c < kv; ++c) {
        const int64_t k = k0 + c;
        if (!p.a_trans)   // A row m of the step: ra(m) + ca(k0) + c
          CHECK(ca[q * p.gk + k0] + c == ca[q * p.gk + k], "A K-step not contiguous in U", k, q);
        if (p.fused_b)    // B row k of the step: rb(k0) + c * ldb
          CHECK(rb[q * p.gk + k0] + c * p.ldb == rb[q * p.gk + k], "B K-step not affine in V", k, q);
      }
    }
  if (gc.dma && !p.a_trans && p.krun == 0) {
    // global-to-LDS tiles: one 128-byte A row per K-step
    const int64_t bkd = 128 / (p.compute == SYMT_COMPUTE_F64 ? 8 : 4);
    CHECK(p.gk % bkd == 0, "DMA tile with a partial K-step", p.gk, bkd);
    for (int q = 0; q < G; ++q)
      for (int64_t k = 0; k < p.gk; ++k) {
        CHECK(ca[q * p.gk + k] == ca[q * p.gk + (k / bkd) * bkd] + k % bkd, "DMA A row not contiguous", k, q);
        if (p.fused_b)
          CHECK(rb[q * p.gk + k] == rb[q * p.gk + (k / bkd) * bkd] + (k % bkd) * p.ldb, "DMA B rows not affine", k, q);
      }
  }
  // vector loads: 16-byte chunks contiguous and aligned (16-byte aligned operands)
  const int vw = p.compute == SYMT_COMPUTE_F64 ? 2 : 4;
  const int64_t run = p.fused_ua ? p.gk : cm * p.nK;
  const bool avec = (p.compute == SYMT_COMPUTE_BF16X3 || run % vw == 0);
  if (avec && !p.a_trans && p.krun == 0)
    for (int q = 0; q < G; ++q)
      for (int64_t m = 0; m < p.M; ++m)
        for (int64_t k = 0; k < p.gk; k += vw)
          CHECK((ra[q * p.M + m] + ca[q * p.gk + k]) % vw == 0, "vector A load misaligned", m, k);
  if (p.a_trans && !p.a_chunks && !p.cplx && p.u_k_run % vw == 0 && p.gk % vw == 0) {
    // K-major A without M chunks on register tiles: 16-byte loads along U's trailing
    // contracted run (rows m, K indices k .. k + vw - 1 at ra(m) + ca(k) + 0 ..)
    ++g_a_kvec;
    for (int q = 0; q < G; ++q)
      for (int64_t k = 0; k < p.gk; k += vw) {
        for (int j = 1; j < vw; ++j)
          CHECK(ca[q * p.gk + k + j] == ca[q * p.gk + k] + j, "K vector of A not contiguous", k, j);
        for (int64_t m = 0; m < p.M; ++m)
          CHECK((ra[q * p.M + m] + ca[q * p.gk + k]) % vw == 0, "K vector of A misaligned", m, k);
      }
  }
  if (p.a_trans && p.a_chunks)
    for (int q = 0; q < G; ++q)
      for (int64_t m = 0; m < p.M; m += vw) {
        for (int j = 1; j < vw && m + j < p.M; ++j)
          CHECK(ra[q * p.M + m + j] == ra[q * p.M + m] + j, "K-major A chunk not contiguous", m, j);
        CHECK(ra[q * p.M + m] % vw == 0, "K-major A chunk misaligned", m, q);
      }
  const int64_t bkd = 128 / (p.compute == SYMT_COMPUTE_F64 ? 8 : 4);
  if (p.a_trans && gc.dma) {
    CHECK(gc.bm == 128 && p.a_chunks, "K-major A on a DMA tile that is not 128 rows or has no chunks", gc.bm,
          p.a_chunks);
    CHECK(p.gk % bkd == 0 && p.M % vw == 0, "K-major A DMA tile with a partial step or chunk", p.gk, p.M);
  }
  if (p.a_trans && p.a_chunks && p.gk % bkd == 0 && p.M % vw == 0) {
    // K-major A on a global-to-LDS tile (the model's choice, or a forced tile):
    // 16-byte chunks along M at every K row's table entry, inside U; the swizzled
    // slots (k, position) hold chunk position ^ ((k & 1) << 3) and the operand
    // reads find element (k, m) there
    ++g_at_dma;
    const int64_t u_n = p.U.elems * cm;
    for (int q = 0; q < G; ++q)
      for (int64_t k = 0; k < p.gk; ++k) {
        CHECK(ca[q * p.gk + k] % vw == 0, "K-major A row misaligned", k, q);
        for (int64_t m = 0; m + vw <= p.M; m += vw) {
          const int64_t a = ca[q * p.gk + k] + ra[q * p.M + m];
          CHECK(a >= 0 && a + vw <= u_n, "K-major A chunk outside U", a, u_n);
        }
      }
    const int ach = 128 / vw;
    std::vector<int> lab(static_cast<size_t>(bkd) * 128, -1);
    for (int slot = 0; slot < bkd * ach; ++slot) {
      const int k = slot / ach, c = (slot % ach) ^ ((k & 1) << 3);
      CHECK(c >= 0 && c < ach, "K-major A swizzle past the row", c, ach);
      for (int e = 0; e < vw; ++e) lab[static_cast<size_t>(slot) * vw + e] = k * 128 + c * vw + e;
    }
    for (int k = 0; k < bkd; ++k)
      for (int m = 0; m < 128; ++m) {
        const int idx = k * 128 + ((m / vw) ^ ((k & 1) << 3)) * vw + m % vw;
        CHECK(lab[idx] == k * 128 + m, "K-major A operand read from the wrong slot", k, m);
      }
  }
  if (p.fused_b && gc.dma && p.krun == 0)
    CHECK(p.fused_b_chunks, "V in place on a DMA tile without whole column chunks", p.gn, p.ldb);
  if (p.fused_b && p.fused_b_chunks)
    for (int q = 0; q < G; ++q)
      for (int64_t n = 0; n < p.gn; n += vw) {
        for (int j = 1; j < vw && n + j < p.gn; ++j)
          CHECK(cb[q * p.gn + n + j] == cb[q * p.gn + n] + j, "B column chunk not contiguous", n, j);
        for (int64_t k = 0; k < p.gk; ++k)
          CHECK((rb[q * p.gk + k] + cb[q * p.gn + n]) % vw == 0, "vector B load misaligned", k, n);
      }
}

// ---------------------------------------------------------------------------
// Stream-K and split K
// ---------------------------------------------------------------------------
void check_stream_k(int64_t batch, int tiles_m, int tiles_n, int nk, int64_t resident, int64_t part_elems,
                    int64_t tile_elems) {
  const int64_t ntiles = batch * tiles_m * tiles_n;
  const SkLaunch sl = sk_launch(ntiles, tiles_n, nk, resident, part_elems, tile_elems, kSkMinIters);
  if (sl.P == 0) return;
  const int P = sl.P, ts = sl.ts;
  CHECK(P % (8 * ts) == 0, "persistent workgroups not whole teams on 8 XCDs", P, ts);
  CHECK(P <= resident, "more persistent workgroups than resident slots", P, resident);
  CHECK(2 * static_cast<int64_t>(P) * tile_elems <= part_elems, "pieces buffer too small", P, part_elems);
  std::vector<uint8_t> cover(static_cast<size_t>(ntiles * nk), 0);
  std::vector<uint8_t> whole(static_cast<size_t>(ntiles), 0);
  std::map<int64_t, std::vector<std::pair<int, int64_t>>> pieces;   // tile -> (kt0, slot)
  std::vector<uint8_t> slot_used(static_cast<size_t>(2 * P), 0);
  for (int b = 0; b < P; ++b) {
    const SkSlot s = sk_slot(b, P, ts);
    CHECK(s.member >= 0 && s.member < ts && s.team >= 0 && s.team < s.nteam, "slot decode", s.team, s.member);
    const int64_t total = ntiles / ts * nk;
    int64_t it = sk_bound(s.team, total, s.nteam);
    const int64_t end = sk_bound(s.team + 1, total, s.nteam);
    const int64_t first = it / nk;
    while (it < end) {
      const int64_t grp = it / nk;
      const int kt0 = static_cast<int>(it - grp * nk);
      const int kt1 = static_cast<int>(std::min<int64_t>(nk, kt0 + (end - it)));
      const int64_t tile = grp * ts + s.member;
      CHECK(tile < ntiles, "tile past the launch", tile, ntiles);
      for (int k = kt0; k < kt1; ++k) {
        CHECK(cover[tile * nk + k] == 0, "K-iteration multiplied twice", tile, k);
        cover[tile * nk + k]++;
      }
      if (kt0 == 0 && kt1 == nk) {
        whole[tile]++;
      } else {
        const int64_t slot = sk_piece(s.team, s.member, ts, grp, first);
        CHECK(slot >= 0 && slot < 2 * P, "piece slot out of range", slot, 2 * P);
        CHECK((slot + 1) * tile_elems <= part_elems, "piece past the buffer", slot, part_elems);
        if (slot >= 0 && slot < 2 * P) {
          CHECK(slot_used[slot] == 0, "piece slot written twice", slot, tile);
          slot_used[slot]++;
        }
        pieces[tile].push_back({kt0, slot});
      }
      it += kt1 - kt0;
    }
  }
  for (int64_t i = 0; i < ntiles * nk; ++i) CHECK(cover[i] == 1, "K-iteration not multiplied", i / nk, i % nk);
  // the fixup, tile by tile
  const int nteam = P / ts;
  const int64_t total = ntiles / ts * nk;
  for (int64_t tile = 0; tile < ntiles; ++tile) {
    const int64_t grp = tile / ts;
    const int member = static_cast<int>(tile - grp * ts);
    const int64_t x0 = grp * nk, x1 = x0 + nk;
    int64_t t = sk_first_team(x0, total, nteam);
    CHECK(sk_bound(t, total, nteam) <= x0 && (t + 1 >= nteam || sk_bound(t + 1, total, nteam) > x0),
          "fixup's first team", t, x0);
    if (sk_bound(t + 1, total, nteam) >= x1) {
      CHECK(whole[tile] == 1 && pieces[tile].empty(), "uncut tile not stored whole once", tile, whole[tile]);
      continue;
    }
    CHECK(whole[tile] == 0, "cut tile also stored whole", tile, 0);
    std::vector<int64_t> got;
    int64_t prev_b0 = -1;
    for (; t < nteam; ++t) {
      const int64_t b0 = sk_bound(t, total, nteam), b1 = sk_bound(t + 1, total, nteam);
      if (b0 >= x1) break;
      if (b1 == b0) continue;
      CHECK(b0 > prev_b0, "fixup not in increasing K order", b0, prev_b0);
      prev_b0 = b0;
      got.push_back(sk_piece(static_cast<int>(t), member, ts, grp, b0 / nk));
    }
    // the kernel lists teams t_first .. t_last (the holder of iteration x1 - 1)
    // in LDS, skipping empty shares: the same pieces in the same order
    const int64_t t_first = sk_first_team(x0, total, nteam), t_last = sk_first_team(x1 - 1, total, nteam);
    CHECK(t_last >= t_first && t_last < nteam, "fixup's last team", t_last, nteam);
    CHECK(sk_bound(t_last, total, nteam) < x1 && (t_last + 1 >= nteam || sk_bound(t_last + 1, total, nteam) >= x1),
          "fixup's last team does not hold iteration x1 - 1", t_last, x1);
    std::vector<int64_t> listed;
    for (int64_t u = t_first; u <= t_last; ++u) {
      const int64_t b0 = sk_bound(u, total, nteam), b1 = sk_bound(u + 1, total, nteam);
      if (b1 > b0) listed.push_back(sk_piece(static_cast<int>(u), member, ts, grp, b0 / nk));
    }
    CHECK(listed == got, "fixup's team list differs from its pieces", tile, static_cast<int64_t>(listed.size()));
    std::vector<int64_t> want;
    auto pc = pieces[tile];
    std::sort(pc.begin(), pc.end());
    for (auto& pr : pc) want.push_back(pr.second);
    CHECK(got == want, "fixup does not read exactly its tile's pieces", tile, static_cast<int64_t>(got.size()));
  }
}

void check_split_k(int64_t ntiles, int splits, int nk_all, int64_t part_elems, int64_t tile_elems) {
  if (splits <= 1) return;
  CHECK(ntiles * splits * tile_elems <= part_elems, "split partial tiles past the buffer", ntiles * splits, part_elems);
  const int per = (nk_all + splits - 1) / splits;
  std::vector<uint8_t> cover(static_cast<size_t>(nk_all), 0);
  for (int sp = 0; sp < splits; ++sp) {
    const int kt0 = std::min(nk_all, sp * per), kt1 = std::min(nk_all, kt0 + per);
    for (int k = kt0; k < kt1; ++k) cover[k]++;
  }
  for (int k = 0; k < nk_all; ++k) CHECK(cover[k] == 1, "split K-step not covered once", k, cover[k]);
}

// ---------------------------------------------------------------------------
// Random contractions
// ---------------------------------------------------------------------------
bool random_case(Rng& rng, Case& c, bool allow_tables, bool allow_sub, bool allow_cplx, int dmax) {
  static const int orders[][3] = {{1, 2, 0}, {1, 3, 0}, {1, 4, 0}, {1, 5, 0}, {2, 2, 2}, {2, 2, 3}, {1, 8, 0},
                                  {1, 6, 0}};
  const auto& og = orders[rng.below(8)];
  c.g = symt_group{};
  c.g.nfactors = og[0];
  c.g.order[0] = og[1];
  if (og[0] == 2) c.g.order[1] = og[2];
  const int G = group_size(c.g);
  int s = rng.below(4), t = rng.below(4), v = rng.below(4);
  if (s + t == 0) s = 1;
  if (s + v > 6 || t + v > 6) return false;
  const char* letters = "abcdefghijkl";
  std::string I(letters, s), K(letters + s, v), J(letters + s + v, t);
  std::string tu = I + K, tv = K + J, tw = I + J;
  auto shuffle = [&](std::string& x) {
    for (int i = static_cast<int>(x.size()) - 1; i > 0; --i) std::swap(x[i], x[rng.below(i + 1)]);
  };
  if (rng.below(3)) shuffle(tu);
  if (rng.below(3)) shuffle(tv);
  if (rng.below(3)) shuffle(tw);
  c.einsum = tu + "," + tv + "->" + tw;
  std::map<char, int64_t> dim;
  std::map<char, int> cu, cv, hs;
  std::map<char, std::vector<int32_t>> tab;
  const bool sub = allow_sub && c.g.nfactors == 1 && rng.below(4) == 0;
  const bool tables = allow_tables && !sub && rng.below(4) == 0;
  for (char m : tu + J) {
    const int r = rng.below(10);
    dim[m] = r < 6 ? 1 + rng.below(dmax) : r < 8 ? 16 * (1 + rng.below(2)) : 1 + rng.below(40);
    if (sub) {
      std::vector<int> div;
      for (int h = 1; h <= G; ++h)
        if (G % h == 0) div.push_back(h);
      hs[m] = div[rng.below(static_cast<int>(div.size()))];
    } else {
      hs[m] = G;
    }
    if (tables) {
      std::vector<int32_t> perm(G);
      std::iota(perm.begin(), perm.end(), 0);
      for (int i = G - 1; i > 0; --i) std::swap(perm[i], perm[rng.below(i + 1)]);
      tab[m] = perm;
    }
  }
  for (char m : tu) cu[m] = rng.coin() ? 1 : -1;
  const int sigma = rng.coin() ? 1 : -1;
  for (char m : tv) cv[m] = K.find(m) != std::string::npos ? sigma * cu[m] : (rng.coin() ? 1 : -1);
  auto fill = [&](Desc& d, const std::string& term, const std::map<char, int>& sg) {
    d.signs.clear();
    d.dims.clear();
    d.tables.clear();
    d.sectors.clear();
    for (char m : term) {
      d.signs.push_back(sg.at(m) > 0 ? '+' : '-');
      d.dims.push_back(dim[m]);
      if (tables) d.tables.insert(d.tables.end(), tab[m].begin(), tab[m].end());
      if (sub) d.sectors.push_back(hs[m]);
    }
    d.charge = rng.below(G);
  };
  fill(c.u, tu, cu);
  fill(c.v, tv, cv);
  // W: derive through the planner (signs, charge); then its tables and sectors
  const bool cplx = allow_cplx && !sub && rng.below(5) == 0;
  c.u.dtype = cplx ? (rng.coin() ? SYMT_C128 : SYMT_C64) : (rng.coin() ? SYMT_F64 : SYMT_F32);
  c.v.dtype = cplx ? (rng.coin() ? SYMT_C128 : SYMT_C64) : (rng.coin() ? SYMT_F64 : SYMT_F32);
  c.u.bind();
  c.v.bind();
  const int cmp = rng.below(3);
  symt_plan_info info;
  std::string err;
  Plan pl;
  if (make_plan(c.einsum.c_str(), &c.g, &c.u.t, &c.v.t, nullptr, cmp, &pl, &err) != SYMT_OK) return false;
  c.w.signs = "";
  for (size_t m = 0; m < tw.size(); ++m) c.w.signs.push_back(pl.w_sign[m] > 0 ? '+' : '-');
  c.w.charge = pl.w_charge;
  c.w.dims.clear();
  c.w.tables.clear();
  c.w.sectors.clear();
  for (char m : tw) {
    c.w.dims.push_back(dim[m]);
    if (tables) c.w.tables.insert(c.w.tables.end(), tab[m].begin(), tab[m].end());
    if (sub) c.w.sectors.push_back(hs[m]);
  }
  const int wt = rng.below(3);
  c.w.dtype = cplx ? (cmp == 1 ? SYMT_C64 : SYMT_C128)
                   : (wt == 0 ? SYMT_F64 : wt == 1 ? SYMT_F32 : (cmp == 1 ? SYMT_F32 : SYMT_F64));
  c.w.bind();
  c.compute = cmp;
  (void)info;
  return true;
}

int64_t elems_of(const Plan& p) { return p.U.elems + p.V.elems + p.W.elems; }

void run_case_once(const Case& c, bool steps) {
  Plan p;
  std::string err;
  const int rc = make_plan(c.einsum.c_str(), &c.g, &c.u.t, &c.v.t, &c.w.t, c.compute | (steps ? kForceSteps : 0),
                           &p, &err);
  if (rc != SYMT_OK) return;
  char buf[160];
  std::snprintf(buf, sizeof buf, "%s G=%d compute=%d steps=%d fused=%d/%d/%d krun=%d at=%d", c.einsum.c_str(),
                p.g.size, c.compute, steps ? 1 : 0, p.fused ? 1 : 0, p.fused_ua ? 1 : 0, p.fused_b ? 1 : 0,
                p.krun, p.a_trans ? 1 : 0);
  g_case = buf;
  check_transforms(p);
  check_fused(p);
  // the product's split K on this shape
  if (p.compute != SYMT_COMPUTE_BF16X3 && p.nq > 0 && p.M > 0 && p.gn > 0 && p.gk > 0) {
    const int elem = p.compute == SYMT_COMPUTE_F64 ? 8 : 4;
    const GemmChoice gc = choose_fp_gemm(p.nq, p.M, p.gn, p.gk, elem, true);
    const int64_t tiles = p.nq * ((p.M + gc.bm - 1) / gc.bm) * ((p.gn + gc.bn - 1) / gc.bn);
    const int spr = p.krun > 0 ? (p.krun + kFpBK - 1) / kFpBK : 0;
    const int nk_all = static_cast<int>(p.krun > 0 ? p.gk / p.krun * spr : (p.gk + kFpBK - 1) / kFpBK);
    check_split_k(tiles, gc.splits, nk_all, static_cast<int64_t>(p.bytes_partial / elem),
                  static_cast<int64_t>(gc.bm) * gc.bn);
  }
}

// Split-bf16 contractions once more on each forced wide tile: their aligned
// planes are then interleaved by K-steps wherever K allows, and the 256 x 256
// tile reads a binary32 U in place where its runs allow.
void run_case(const Case& c, bool steps) {
  run_case_once(c, steps);
  if (c.compute != SYMT_COMPUTE_BF16X3) return;
  for (const char* tile : {"bw256x256s2", "bw256x128s3"}) {
    setenv("SYMT_GEMM_TILE", tile, 1);
    run_case_once(c, steps);
  }
  unsetenv("SYMT_GEMM_TILE");
}

// The workloads' own shapes (small enough to walk element by element).
void workload_cases() {
  struct W {
    const char* sub;
    int G;
    const char *su, *sv;
    std::vector<int64_t> du, dv;
  };
  const std::vector<W> ws = {
      {"abkl,klij->abij", 4, "++--", "++--", {4, 4, 4, 4}, {4, 4, 4, 4}},
      {"abcd,cdij->abij", 8, "++--", "++--", {6, 6, 6, 6}, {6, 6, 3, 3}},
      {"abc,asA->bcsA", 6, "---", "++-", {8, 4, 8}, {8, 2, 8}},
      {"bcsA,bsSB->cASB", 6, "--+-", "+---", {4, 8, 2, 8}, {4, 2, 2, 4}},
      {"cASB,cSC->ABC", 6, "----", "++-", {8, 8, 2, 4}, {8, 2, 8}},
      // the chain's gradient with respect to W: a long-K product whose K runs (A)
      // hold whole 16-deep groups
      {"bcsA,cASB->bsSB", 6, "--+-", "----", {2, 8, 2, 16}, {8, 16, 2, 2}},
      {"opij,opkm->ijmk", 8, "++--", "--++", {3, 3, 4, 4}, {3, 3, 4, 2}},
      // the ladder's form with K a whole number of 32-deep steps and U's runs of 4
      // and 16 (split-bf16 on the wide tiles, U in place)
      {"abcd,cdij->abij", 8, "++--", "++--", {3, 5, 2, 2}, {2, 2, 4, 9}},
      {"abkl,klij->abij", 4, "++--", "++--", {9, 8, 4, 4}, {4, 4, 5, 13}},
      {"ijk,klm->ijlm", 5, "++-", "++-", {7, 10, 7}, {7, 1, 7}},
  };
  for (const W& w : ws) {
    Case c;
    c.einsum = w.sub;
    c.g.nfactors = w.G == 6 ? 2 : 1;
    c.g.order[0] = w.G == 6 ? 2 : w.G;
    if (w.G == 6) c.g.order[1] = 3;
    c.u.signs = w.su;
    c.v.signs = w.sv;
    c.u.dims = w.du;
    c.v.dims = w.dv;
    c.u.bind();
    c.v.bind();
    Plan pl;
    std::string err;
    for (int cmp = 0; cmp < 3; ++cmp) {
      if (make_plan(c.einsum.c_str(), &c.g, &c.u.t, &c.v.t, nullptr, cmp, &pl, &err) != SYMT_OK) {
        g_case = w.sub;
        fail("workload does not plan", cmp, 0);
        continue;
      }
      c.w.signs.clear();
      const std::string tw = c.einsum.substr(c.einsum.find("->") + 2);
      for (size_t m = 0; m < tw.size(); ++m) c.w.signs.push_back(pl.w_sign[m] > 0 ? '+' : '-');
      c.w.charge = pl.w_charge;
      c.w.dims.assign(pl.W.dims, pl.W.dims + pl.W.n);
      c.w.dtype = cmp == 1 ? SYMT_F32 : SYMT_F64;
      c.w.bind();
      c.compute = cmp;
      for (int dt = 0; dt < 2; ++dt) {
        c.u.dtype = c.v.dtype = dt ? SYMT_F32 : SYMT_F64;
        c.u.bind();
        c.v.bind();
        run_case(c, false);
        run_case(c, true);
      }
    }
  }
}

}  // namespace

int main(int argc, char** argv) {
  const int n = argc > 1 ? std::atoi(argv[1]) : 400;
  const uint64_t seed = argc > 2 ? std::strtoull(argv[2], nullptr, 10) : 20070805ull;
  workload_cases();
  Rng rng{seed};
  int done = 0;
  while (done < n) {
    Case c;
    if (!random_case(rng, c, true, true, true, 6)) continue;
    Plan p;
    std::string err;
    if (make_plan(c.einsum.c_str(), &c.g, &c.u.t, &c.v.t, &c.w.t, c.compute, &p, &err) != SYMT_OK) continue;
    if (elems_of(p) > 400000) continue;        // keep the element walks quick
    run_case(c, false);
    run_case(c, rng.below(3) == 0);
    ++done;
  }
  // stream-K partitions over launch shapes, including the workloads' (Z_8 and
  // Z_16 ladders on 96 x 96 tiles, the MPS chain's products)
  g_case = "stream-K";
  const int64_t resident[] = {256, 512, 768};
  for (int64_t res : resident)
    for (int64_t batch : {1, 2, 6, 8, 16})
      for (int tm : {1, 2, 3, 5, 16, 48})
        for (int tn : {1, 2, 3, 4, 11, 16})
          for (int nk : {1, 3, 4, 7, 16, 36, 97, 288})
            for (int64_t te : {96 * 96, 128 * 128}) {
              check_stream_k(batch, tm, tn, nk, res, 2 * res * te, te);
              check_stream_k(batch, tm, tn, nk, res, 2 * res * te - 1, te);   // a buffer one short
            }
  check_stream_k(8, 48, 3, 288, 768, 2 * 768 * 96 * 96, 96 * 96);          // Z_8 ladder (f64, K = 4608)
  check_stream_k(16, 171, 11, 1024, 768, 2 * 768 * 96 * 96, 96 * 96);      // Z_16 ladder (f64, K = 16384)
  g_case = "split-K";
  for (int64_t tiles : {1, 2, 5, 64, 300})
    for (int sp : {2, 3, 8, 64, 128})
      for (int nk : {8, 16, 17, 100, 185193})
        check_split_k(tiles, sp, nk, tiles * sp * 128 * 128, 128 * 128);
  std::printf("host replay: %d random contractions + workload shapes, %lld checks (%lld global-to-LDS long-K"
              " plans, %lld with K-major A for global-to-LDS tiles, %lld with row vectors, %lld with K vectors of K-major"
              " A, %lld with K vectors on rows, %lld interleaved split-bf16 plane transforms, %lld split-bf16 plans reading U"
              " in place on the wide tile), %d failures\n", done, static_cast<long long>(g_checks),
              static_cast<long long>(g_tallk_dma), static_cast<long long>(g_at_dma), static_cast<long long>(g_row_vec),
              static_cast<long long>(g_a_kvec), static_cast<long long>(g_k_vec), static_cast<long long>(g_bf16_il),
              static_cast<long long>(g_bf16_fa), g_failures);
  return g_failures == 0 ? 0 : 1;
}

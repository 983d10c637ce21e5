// Host-side plan of one symmetric contraction and the POD descriptors handed to
// the transform and sector-product kernels.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "symtensor.h"

namespace symt {

constexpr int kMaxOrder = SYMT_MAX_ORDER;
constexpr int kMaxDims = SYMT_MAX_ORDER + 1;

struct GroupDesc {
  int32_t nf;                       // number of cyclic factors
  int32_t ord[SYMT_MAX_FACTORS];    // factor orders, first most significant
  int32_t size;                     // |G|
};

// One sector group of an aligned operand (rows or columns of its matrix form).
// The sectors S[pos[i]] of the group's modes obey
//     sum_i coef[i] * S[pos[i]] == alpha * Q + beta      (in G)
// which is one of the three generalized Kronecker deltas of Alg. 2
// (delta(1) on I, delta(2) on K, delta(3) on J).  The last listed mode is the
// implicit one; the others are stored, first most significant.
struct SectorGroup {
  int32_t count;
  int32_t pos[kMaxOrder];
  int32_t coef[kMaxOrder];          // sign of each member's coefficient
  int32_t rad[kMaxOrder];           // sectors of each member (|G|, or H for a subgroup mode)
  int32_t mag[kMaxOrder];           // |G| / rad: the coefficient's magnitude
  int32_t alpha;
  int32_t beta;
};

// Layout variants of an aligned matrix (|G|, rows, cols).
enum AlignedLayout : int32_t {
  kRowMajor = 0,     // [Q][row][col]
  kColMajor = 1      // [Q][col][row]  (row index fastest)
};

// Element types the transform moves between.
enum XType : int32_t { kXF64 = 0, kXF32 = 1, kXBF16Split = 2 };

// Everything one transform launch needs; passed to the kernel by value.
struct XformParams {
  GroupDesc g;
  int32_t order;                    // modes of the operand
  SectorGroup row, col;
  int64_t gpow_row, gpow_col;       // stored-sector tuples of each group (product of radices)
  int32_t hs[kMaxOrder];            // sectors of each mode of the operand (standard block index radices)
  int64_t nblocks;                  // aligned blocks moved: slices x stored-sector tuples
  int32_t q0, q_step;               // auxiliary sectors moved: Q = q0 + q_step * slice
  int32_t q_full;                   // 1: the aligned buffer holds all |G| slices (offset by Q);
                                    // 0: only the moved slices, in order (offset by slice)
  int64_t blk_elems;                // elements per block (product of inner dims)
  int64_t q_stride, rs_stride, cs_stride;  // aligned block base = Q*q + Rs*rs + Cs*cs
  int64_t plane;                    // elements between the hi and lo bf16 planes
  int32_t il;                       // split-bf16 destination interleaved by 32-deep K-steps:
                                    // hi of aligned offset o at 2 o - o % 32, lo `plane` (32) after
  int32_t to_aligned;               // 1: standard -> aligned, 0: aligned -> standard
  // inner dims after merging; src / dst strides already oriented by direction
  int32_t mode;                     // 0 copy (one run dim), 1 tiled transpose
  int32_t run;                      // copy: run dim
  int64_t run_len;                  // copy: size[run]; transpose: elements of the A index
  int64_t run_ss, run_ds;           // copy: strides of the run dim
  int64_t t_len;                    // transpose: elements of the B index
  // Transpose tile indices, each a mixed-radix merge of dims listed fastest
  // first: A (read along, smallest source strides) and B (written along,
  // smallest destination strides among the rest).
  int32_t na, nb;
  int64_t asize[kMaxDims], ass[kMaxDims], ads[kMaxDims];
  int64_t tsize[kMaxDims], tss[kMaxDims], tds[kMaxDims];
  int32_t nbatch;                   // remaining dims ("rows")
  int64_t bsize[kMaxDims];
  int64_t bss[kMaxDims];
  int64_t bds[kMaxDims];
  int64_t rows;                     // product of bsize
  int64_t rows_per_tile;            // copy: rows per workgroup
  int64_t run_chunk, run_tiles;     // copy: run elements per workgroup, chunks per run
  int64_t tiles_per_block;          // workgroups per block
  int32_t lanes_per_row;            // copy: power of two <= 64
  int32_t lanes_log2;
  int32_t vec;                      // elements per thread access along the run (1, 2, 4)
  int32_t tiles_run, tiles_t;       // transpose: tiles along run and tdim
  int32_t tr_write;                 // transpose: lanes write the tile's A side in
                                    // destination order (A holds the destination's
                                    // fastest dims; B's are strided)
  const int32_t* chg;               // device charge tables of the operand, or nullptr (identity)
};

// Offsets of one sector group of an aligned operand inside its standard
// reduced form.  The standard-form offset of aligned element (Q, r, c) splits
// as R(Q, r) + C(Q, c): the block index and the in-block offset are both
// linear in the sectors and in-block indices, and every sector (stored or
// implicit) belongs to exactly one group.  One OffsetParams describes R or C.
struct OffsetParams {
  GroupDesc g;
  SectorGroup grp;                  // the group's modes, coefficients and delta
  int64_t gpow;                     // |G|^(count-1): stored sector combinations
  int64_t n_inner;                  // product of the group's inner dims
  int64_t count;                    // entries per Q = gpow * n_inner (x 2 with pairs)
  int32_t scale;                    // reals per element: 2 for complex operands, else 1
  int32_t pairs;                    // 1: column table of a complex operand, entry 2c + comp
  int64_t dim[kMaxOrder];           // inner dims of the group's modes (group order)
  int64_t stride[kMaxOrder];        // their standard-form strides
  int64_t weight[kMaxOrder];        // standard-form offset of one unit of each mode's sector
  const int32_t* chg;               // device charge tables of the operand, or nullptr (identity)
  // affine = 1: entry (q, i) = q * aff_q + i * aff_i (the tables of an aligned form)
  int32_t affine;
  int64_t aff_q, aff_i;
};

// Up to six offset tables filled by one launch (entries of table t:
// out[t][q * count + i] for q < |G|).
constexpr int kMaxOffsetTables = 6;
struct OffsetBatch {
  int32_t n = 0;
  OffsetParams t[kMaxOffsetTables];
  int64_t* out[kMaxOffsetTables];
  int64_t end[kMaxOffsetTables];    // running sum of |G| * count
};

// Both descriptors travel as kernel arguments (at most 4 KB).
static_assert(sizeof(OffsetBatch) <= 4000, "offset batch exceeds the kernel argument space");
static_assert(sizeof(XformParams) <= 4000, "transform descriptor exceeds the kernel argument space");

// Device pointers of the offset tables of the fused product: rows and columns
// of U (A operand) and of W (output), each |G| x (rows or columns); with rb set,
// also V's (B read in place: row k0 + k of a K-step at rb[k0] + k * ldb).
struct FusedTables {
  const int64_t* ra;
  const int64_t* ca;
  const int64_t* rc;
  const int64_t* cc;
  int32_t vec;                      // 1: U is not 16-byte aligned, load A one element at a time
  const int64_t* rb = nullptr;      // nullptr: B is the aligned V_al
  const int64_t* cb = nullptr;
  int64_t ldb = 0;
  int32_t a_bytes = 8;              // split-bf16 product: U's element size (8 binary64, 4 binary32)
  int32_t krun = 0;                 // > 0: K stepped run by run (register tiles)
  int32_t c_bytes = 8;              // split-bf16 products: W's element size (8 binary64, 4 binary32)
  int32_t at = 0;                   // 1: A loaded K-major from U (register tiles)
  int32_t c_trans = 0;              // 1: W's rows are its contiguous index (row-streaming product)
  int32_t a_klanes = 0;             // 1: U's K index runs contiguous for 16 or more (long-K product)
  int32_t c_rows4 = 0;              // 1: W's rows in contiguous runs of a multiple of 4 elements
  int32_t a_kvec = 0;               // 1 (K-major A without M chunks): U 16-byte aligned, its contracted
                                    //    modes ending in runs of 16 bytes, B's loads vectors too
  int32_t a_krow = 0;               // 1 (A not K-major): A's K index contiguous in 16-byte aligned runs
  int32_t k_groups = 0;             // 1: every 16-deep group of K lies in one run of A's rows and one
                                    //    affine run of B's rows, B's columns in 16-byte chunks (long-K)
};

struct OperandDesc {
  int32_t n;                        // order
  int32_t sign[kMaxOrder];          // +1 / -1
  int32_t charge;
  int64_t dims[kMaxOrder];
  int32_t hs[kMaxOrder];            // sectors per mode: |G|, or H | |G| for a subgroup mode
  int32_t dtype;
  void* data;
  int64_t elems;                    // elements of the standard reduced form
};

struct Plan {
  GroupDesc g;
  std::string tu, tv, tw;
  int32_t s = 0, t = 0, v = 0, sigma = 0;
  int32_t q_pin = -1;               // s, t or v = 0: the one auxiliary sector with nonzero blocks
  // auxiliary sectors for which all three deltas can hold (a coset q0 + q_step Z of Z_G,
  // nq of them): the slices the contraction aligns, multiplies and writes back
  int32_t q0 = 0, q_step = 1;
  int64_t nq = 0;
  int32_t posI_u[kMaxOrder], posK_u[kMaxOrder], posK_v[kMaxOrder], posJ_v[kMaxOrder];
  int32_t posI_w[kMaxOrder], posJ_w[kMaxOrder];
  int64_t nI = 1, nK = 1, nJ = 1;
  int64_t M = 0, Kd = 0, N = 0;
  bool cplx = false;                // complex operands: the product runs on C's real representation
  bool subgroups = false;           // some mode has fewer than |G| sectors
  int64_t gk = 0, gn = 0;           // the real product's K and N (2 Kd, 2 N when complex)
  int64_t kpad = 0;                 // split-bf16: K pitch of the contraction's workspace
                                    // planes (gk rounded up to 8; the pad is zero), else gk
  OperandDesc U, V, W;
  bool has_w = false;
  int32_t w_sign[kMaxOrder];        // derived
  int32_t w_charge = 0;             // derived
  int32_t compute = 0;
  bool fused = false;               // A read from U's standard form, C written to W's
  // fused product on U_al: U's contracted modes are not its last ones (or its runs
  // do not suit the product's tiles), so U is aligned first; B and C as when fused
  bool fused_ua = false;
  // split-bf16 workspace planes interleaved by 32-deep K-steps (a row's hi and lo
  // halves of one K-step share a 128-byte line): both operands aligned and the
  // product on the wide tiles
  bool bf16_il = false;
  // ... and U (binary32, its contracted modes last in runs of 4) read in place by
  // the 256 x 256 wide tile, split when its fragments are read (where U is
  // 16-byte aligned; else U is aligned first as for fused_ua)
  bool bf16_wide_fa = false;
  // fused with A loaded K-major (U's contracted modes are not its last ones): row k
  // of a K-step at ca(Q, k), M chunks at ra(Q, m); a_chunks: U's other modes come
  // in runs of whole 16-byte chunks (vector loads along M)
  bool a_trans = false;
  bool a_chunks = false;
  // B read from V's standard form too (no V_al): V's rows are affine inside every
  // K-step (stride ldb) and its columns come in runs of whole 16-byte chunks
  // (used when V is 16-byte aligned)
  bool fused_b = false;
  bool fused_b_chunks = false;      // V's columns in whole 16-byte chunks
  int64_t ldb = 0;
  // W's contiguous runs at its end: of its output modes from V (columns of the
  // product) and of those from U (rows); one of them is 1
  int64_t w_col_run = 1, w_row_run = 1;
  int64_t u_k_run = 1;              // U's contiguous run of its contracted index (in elements)
  // fused with K runs that do not hold whole K-steps: the register tiles step each
  // run on its own (krun = the run length; 0 = plain K-steps)
  int32_t krun = 0;
  size_t bytes_u_al = 0, bytes_v_al = 0, bytes_w_al = 0, workspace = 0;
  size_t ws_u_al = 0, ws_v_al = 0, ws_w_al = 0;   // their regions in the contraction's workspace
  size_t bytes_tables = 0;          // fused (or fused_ua): four offset tables, six with fused_b
  size_t bytes_partial = 0;         // stream-K pieces of the product (0: data-parallel tiles)
  // Charge tables (label -> charge) of U, V, W, n x |G| each; empty = identity.
  // On the device each operand's block is [mode][label -> charge | charge -> label][|G|].
  std::vector<int32_t> chg[3];
  bool charges = false;             // some table is not the identity
  size_t bytes_charges = 0;         // device copy of all three (0 when charges is false)
  double flops = 0.0;
};

// Whether V's standard form can serve as the product's B operand directly
// (affine rows inside every K-step, 16-byte column chunks); *ldb = row stride,
// *chunks = whether its columns come in whole 16-byte chunks (needed for vector
// loads of B when K is stepped run by run).
bool v_in_place_layout(const Plan& p, int64_t* ldb, bool* chunks = nullptr);

// Parse and validate; returns a SYMT_* status and fills `err` on failure.
int make_plan(const char* einsum, const symt_group* group, const symt_tensor* u,
              const symt_tensor* v, const symt_tensor* w, int32_t compute, Plan* plan,
              std::string* err);

// Bit of the compute argument that forces the three separate steps.
constexpr int32_t kForceSteps = 0x100;
// K-depth of every f64/f32 product tile (the fused path needs contiguous runs of it).
constexpr int kFpBK = 16;

// Launch choice of the f64 / f32 sector product, from a host-side cost model.
struct GemmChoice {
  int tile = -1;              // row of the tile table (dispatch order of the launcher)
  int bm = 0, bn = 0;
  bool dma = false;           // global-to-LDS tile
  bool sk = false;            // stream-K: persistent workgroups split the K-iterations of all
                              // tiles evenly; tiles cut between two of them are summed after
  int splits = 1;             // register tiles: each tile's K-steps in this many runs, summed after
  size_t partial_bytes = 0;   // workspace for stream-K pieces or split partial tiles
};
// Most persistent workgroups of a stream-K product: 256 CUs x up to 3 resident
// workgroups (the two-stage 96 x 96 tile).  The planner sizes the pieces
// buffer (two pieces per workgroup) from each tile's resident workgroups; a
// launch runs no more workgroups than that buffer holds.
constexpr int kSkSlots = 768;
// GemmChoice::tile of the row-streaming product (K and N at most 64, many rows):
// past the tile table.
constexpr int kRowsTile = 64;
// GemmChoice::tile of the long-K product with M and N at most 64 (GemmChoice::
// splits = its K ranges per slice, partial_bytes = their partial outputs).
constexpr int kTallKTile = 65;
// K ranges per slice of the long-K product (at most two workgroups per CU over
// all slices, so that whole rounds of one or two resident workgroups per CU
// cover them; at least 256 K indices each) and the K indices of each range (a
// multiple of 16, the last range shorter or empty).
inline int tallk_ranges(int64_t batch, int64_t K) {
  const int64_t want = 512 / (batch > 0 ? batch : 1);
  const int64_t most = (K + 255) / 256;
  const int64_t r = want < most ? want : most;
  return static_cast<int>(r < 1 ? 1 : r);
}
inline int tallk_range(int64_t K, int ranges) {
  const int64_t per = (K + ranges - 1) / ranges;
  return static_cast<int>((per + 15) / 16 * 16);
}
// Whether the fused product's operands hold the long-K product's 16-deep groups
// of K (FusedTables::k_groups): A's K runs (U_al rows, or U's trailing
// contracted run) and V's contracted runs are whole groups, V's columns whole
// 16-byte chunks (V in place) or V_al's rows a whole number of chunks.
bool tallk_groups(const Plan& p);
// Fewest K-iterations a stream-K workgroup takes on (bounds the pieces per tile).
constexpr int kSkMinIters = 4;
// a_kmajor: A is read K-major from U (global-to-LDS tiles of 128 rows only).
GemmChoice choose_fp_gemm(int64_t batch, int64_t M, int64_t N, int64_t K, int elem, bool aligned,
                          bool a_kmajor = false);
// Split-bf16 product: whether the launcher runs register-staged tiles on this
// shape (else global-to-LDS ones), and which of the fused product's three
// register tiles it takes (0: 128 x 64, 1: 128 x 128, 2: 128 x 256, 3: 128 x 96).
bool bf16x3_register_tile(int64_t M, int64_t N, int64_t K);
int bf16x3_fused_tile(int64_t M, int64_t N);
// Wide split-bf16 tile of the global-to-LDS product on bf16 planes (0: 256 x 256,
// 1: 256 x 128, one binary32 accumulator), or -1 where N pads by more than an
// eighth or the launch has fewer tiles than the device has CUs.
int bf16x3_wide_tile(int64_t batch, int64_t M, int64_t N);

// True when the aligned form of operand 0 (U), 1 (V) or 2 (W) is zero outside
// slice q_pin: U_al carries deltas (1) and (2), V_al (2) and (3), W_al is their
// product.
inline bool pinned_form(const Plan& p, int operand) {
  if (p.q_pin < 0) return false;
  return operand == 0 ? (p.s == 0 || p.v == 0) : operand == 1 ? (p.t == 0 || p.v == 0) : true;
}

// Transform descriptor for operand 0 (U), 1 (V) or 2 (W) in the given direction.
// `in_elem_bytes` / `out_elem_bytes` are the element sizes of the source and
// destination.  `slice_only`: with Q pinned, the aligned side is the one nonzero
// slice (the contraction's workspace) rather than the full |G|-slice form.
XformParams make_xform(const Plan& p, int operand, bool to_aligned, int in_elem_bytes,
                       int out_elem_bytes, bool out_is_split, bool slice_only);

// Row (rows = true) or column offset table of operand 0 (U), 1 (V) or 2 (W).
OffsetParams make_offsets(const Plan& p, int operand, bool rows);
// Table of an aligned form held in order: entry (q, i) = q * per_q + i * step,
// `count` entries per Q.
OffsetParams affine_offsets(const Plan& p, int64_t count, int64_t per_q, int64_t step);

// Complex storage dtype, and bytes of one real component of an element.
inline bool is_complex(int32_t dtype) { return dtype == SYMT_C128 || dtype == SYMT_C64; }
inline int real_bytes(int32_t dtype) { return dtype == SYMT_F64 || dtype == SYMT_C128 ? 8 : 4; }

// Aligned layout used for an operand under a compute mode.
AlignedLayout aligned_layout(int32_t compute, int operand);

size_t round_up(size_t x, size_t a);

// Device layout of the charge tables of all three operands (forward and
// inverse per mode); `offset[op]` is each operand's first int32.
std::vector<int32_t> charge_tables_device(const Plan& p, int64_t offset[3]);

}  // namespace symt

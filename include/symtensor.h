/*
 * symtensor.h -- C ABI of the irreducible-representation-alignment contraction
 * for tensors with cyclic-group (Z_G) or product-of-cyclic-group symmetry,
 * built for AMD Instinct MI355X (gfx950).
 *
 * The method (Gao, Helms, Chan, Solomonik, "Automatic transformation of
 * irreducible representations for efficient contraction of tensors with cyclic
 * group symmetry"):
 *   (a) each operand's standard reduced form is remapped into an aligned
 *       reduced form indexed by an auxiliary sector Q (Sec. 2.1 "aligned"
 *       maps; Alg. 2, aligned-operand step);
 *   (b) one dense product per Q value contracts the aligned forms (Sec. 2.1,
 *       einsum "AQL,LQJ->AQJ"; Alg. 2, product step);
 *   (c) the aligned output is remapped to the standard reduced form of W
 *       (Alg. 2, final step).
 *
 * Tensor model (Sec. 2.2, Eq. symtsr).  An order-N operand has modes
 * m = 0..N-1, each with |G| sectors and a block (inner) dimension n_m.  With
 * coefficients c_m in {+1,-1} (the sign string) and a total charge Z, element
 * (I_0 i_0, ..., I_{N-1} i_{N-1}) may be nonzero only if
 * sum_m c_m I_m == Z in G.  G = Z_{g_1} x ... x Z_{g_f}; a group element is an
 * int in [0,|G|), mixed radix with the first factor most significant, added
 * component-wise.  The STANDARD REDUCED FORM is the row-major array
 *     [|G|]^(N-1) x n_0 x n_1 x ... x n_{N-1}
 * holding the sectors of modes 0..N-2 and every in-block index; the sector of
 * mode N-1 is the one the rule implies (layout of the API example, Sec. 3).
 *
 * Contractions (Eq. ctr).  "tu,tv->tw" with one letter per mode.  Letters of
 * tu also in tw form I (s modes), of tu also in tv form K (v contracted
 * modes), of tv also in tw form J (t modes).  Every letter sits in exactly two
 * terms; s, t, v >= 1.  The contracted modes must carry the same coefficient
 * ratio sigma = c^V_k / c^U_k for every k (sigma = +1 is Alg. 2's assumption;
 * sigma = -1 is the worked example of Sec. 2.1).  The output's rule is then
 * c^W = (c^U_I, -sigma c^V_J) in tw order and Z^W = Z^U - sigma Z^V (proof of
 * Sec. 2.3); (c^W, Z^W) and (-c^W, -Z^W) are the same rule and both are
 * accepted.
 *
 * ALIGNED LAYOUTS (produced by step (a), consumed by (b), fixed by this ABI).
 * Group orders: I and K in tu order, J in tv order.  The implicit (unstored)
 * sector of each group is its last mode.  Q = sum_{k in K} c^U_k K_k.
 *   U_al[Q][I stored sectors][I inner][K stored sectors][K inner]  -> (|G|, M, Kd)
 *   V_al[Q][K stored sectors][K inner][J stored sectors][J inner]  -> (|G|, Kd, N)
 *   W_al[Q][I stored sectors][I inner][J stored sectors][J inner]  -> (|G|, M, N)
 * with M = |G|^(s-1) prod n_I, Kd = |G|^(v-1) prod n_K, N = |G|^(t-1) prod n_J
 * (with subgroup modes each |G| factor is the stored mode's sector count H_m;
 * aligned blocks whose implicit sector has no solution are zero).
 * Implicit sectors: last I from sum c^U_I I + Q == Z^U; last K from
 * sum c^U_K K == Q; last J from sum c^V_J J + sigma Q == Z^V.
 * Per compute mode the aligned buffers hold:
 *   SYMT_COMPUTE_F64    U_al f64 (|G|,M,Kd) row-major; V_al f64 (|G|,Kd,N); W_al f64 (|G|,M,N)
 *   SYMT_COMPUTE_F32    the same shapes in f32
 *   SYMT_COMPUTE_BF16X3 U_al = two bf16 planes hi then lo, each (|G|,M,Kd);
 *                       V_al = two bf16 planes hi then lo, each (|G|,N,Kd) (Kd fastest);
 *                       W_al f64 (|G|,M,N).
 *   hi = bf16(x), lo = bf16(x - hi), x taken in binary32, both rounded to
 *   nearest even; the product is hi*hi + hi*lo + lo*hi with binary32
 *   accumulation (two accumulators) and a binary64 sum of the two at the end.
 *
 * COMPLEX OPERANDS (Sec. 2.2 allows tensors over C).  u, v and w are all
 * complex (SYMT_C128 / SYMT_C64) or all real, else SYMT_EDTYPE; any compute
 * mode.  The product runs on the real representation of C: with Kd and N the
 * complex extents,
 *   U_al  real (|G|, M, 2 Kd): the (re, im) pair of column k at 2k, 2k + 1;
 *   V_al  real (|G|, 2 Kd, 2 N): row 2k holds (re, im) of V's row k, row
 *         2k + 1 holds (-im, re), pairs at columns 2n, 2n + 1 (BF16X3: the
 *         hi and lo planes of the same real matrix stored (|G|, 2 N, 2 Kd),
 *         the split of -im being minus the split of im);
 *   W_al  real (|G|, M, 2 N): (re, im) of W's column n at 2n, 2n + 1;
 * so the real product U_al V_al is the complex one.  symt_plan_info reports
 * this real product (k = 2 Kd, n = 2 N, flops = 8 |G| M Kd N).  The fused
 * product (below) reads u's and writes w's (re, im) pairs as reals (F64 and
 * F32; BF16X3 runs complex contractions in three steps).
 *
 * EMPTY MODE GROUPS (s, t or v = 0; Sec. 2.1's deltas with an empty sum).  One
 * delta then fixes Q on its own: v = 0 (an outer product) gives Q = 0 and
 * sigma is taken as -1 (W's rule then lists u's coefficients and v's, with
 * Z^W = Z^U + Z^V), or as +1 when a given w carries the rule derived with +1
 * and not the -1 one (an outer product's nonzero blocks obey u's and v's rules
 * each on its own, so both rules describe them: the gradient dU = dW (x) V of
 * a contraction whose only contracted modes are all of V's is such a case);
 * s = 0 gives Q = Z^U; t = 0 gives Q = sigma Z^V.
 * The forms that carry that delta are zero outside that slice: U_al when s or
 * v is 0, V_al when t or v is 0, and W_al always.  symtensor_align writes the
 * whole form, zeros included; symtensor_contract only needs and multiplies the
 * one slice (its workspace holds one slice of each form).  With v = 0 the
 * derived rule of W also admits blocks that break u's own rule; they are
 * written as zeros.
 *
 * FUSED PRODUCT.  The standard-form offset of aligned element (Q, r, c) of any
 * operand splits as R(Q, r) + C(Q, c) (the block index and the in-block offset
 * are linear in the sectors and indices, and each implicit sector belongs to one
 * sector group).  symtensor_contract uses this when compute is F64 or F32, u is
 * stored in the compute type (complex: its complex counterpart), w too, no mode
 * is a subgroup mode, every Q slice is live and u's last v modes are exactly its
 * contracted modes (or see K-major A below).  It builds the offset tables of U and W (once per
 * cached plan, on the context; see Execution and ownership; else in the workspace)
 * and runs one product that reads A straight from u's standard form and writes
 * C straight into w's, so U_al and W_al are never materialised
 * (info.fused = 1).  A K run (u's contracted block, in reals) that holds whole
 * K-steps of the product (16 reals, and 16 f64 / 32 f32 on the global-to-LDS
 * tiles), or is all of K, is stepped as usual; any other run length is stepped
 * run by run (the last step of each run masked at its end) on register-staged
 * tiles, real operands only, where the product would run on them anyway: the
 * sums are then grouped differently from the three-step path's (within the
 * same error bound).  With compute BF16X3 the fused product needs u in binary64
 * or binary32, w in binary64 or binary32 (the binary64 sums rounded on the
 * store, as the W transform rounds them), K runs of whole 32-deep K-steps and a shape on
 * register-staged tiles (not the global-to-LDS ones the product takes from
 * 256 x 512 up): it then splits u's elements into hi/lo in registers, giving
 * the same bits as the hi/lo planes.  V is aligned as usual, unless v is real
 * and in the compute type and its contracted modes are affine in u's K order
 * (each one's stride is the next one's stride times its block size), with
 * whole K-steps per K run and output modes last whose contiguous run is a
 * multiple of 16 bytes (or K stepped run by run), and v is 16-byte aligned
 * (or K stepped run by run): then two more tables let the product read B from
 * v's standard form as well (info.fused_v = 1) and no aligned form is written
 * at all.  Where u's contracted modes are not its last ones, u and w are real
 * and in the compute type and the product runs on register-staged tiles, or on
 * 128-row global-to-LDS tiles with u's trailing output modes in whole 16-byte
 * chunks (and u 16-byte aligned; else a register-staged tile takes over), A is
 * loaded K-major straight from u (each row of a K-step from its own table
 * entry, chunks along u's other modes), with the same values in the same order
 * (info.fused = 1).  Where u does not qualify otherwise (other global-to-LDS
 * shapes, or runs that suit neither stepping), compute is F64 or F32, the operands
 * are real, w is in the compute type, no mode is a subgroup mode and every Q
 * slice is live, u alone is aligned first and the same product reads U_al
 * through affine tables (info.fused = 0, info.fused_w = 1); with BF16X3, u and
 * v go to their hi/lo planes and only w is written in place, where w (binary64
 * or binary32) takes its product columns in contiguous runs of 16 or more.  On
 * the wide split-bf16 tiles (products from 256 x 256 with K a multiple of 32)
 * the planes are interleaved by 32-deep K-steps, and a binary32 u whose
 * contracted modes are its last ones, in runs of 4 or more elements per block,
 * 16-byte aligned, is read in place by the 256 x 256 tile and split in
 * registers (same bits as its planes).  The workspace holds
 * U_al in that case (left unused when u is read in place), then V_al (used when
 * v is not read in place) and the tables.  Where K-steps are the three-step path's, results are identical in
 * value to it: the product sums in the same order.
 *
 * Execution and ownership.  Every device buffer the caller names (operand
 * data, workspace, aligned buffers) is allocated and owned by the caller.  A
 * context holds the HIP device, timing events, the last error and a cache of
 * the plans it has made (keyed by every planning input except data pointers,
 * guarded by a mutex).  Its one device allocation: symtensor_contract keeps
 * each cached plan's fused-product offset tables (they depend on the plan
 * only) in device memory of its own, built on the stream of the plan's first
 * call and awaited through an event by later calls on other streams; at most
 * 1 GiB per context, freed when the cache is cleared (1024 plans) or the
 * context destroyed (freeing waits for the device).  On a stream under graph
 * capture, beyond that budget or when the allocation fails, the tables are
 * built in the workspace on every call instead (the workspace size does not
 * change).  symtensor_contract_static never allocates.  Functions taking a stream
 * (a hipStream_t passed as void*, NULL = the null stream) enqueue their
 * kernels on it and return without synchronising.  All validation happens on
 * the host before the first launch: on any error no kernel is launched and no
 * output byte is written.  A kernel fault surfaces at the caller's next
 * synchronisation.  A context must not be used by two threads at once.
 *
 * Return values: SYMT_OK (0) or one of the negative codes below; the detail of
 * the last failure on a context is in symtensor_last_error().
 *
 * Environment (read at planning and launch time; for tuning and tests only,
 * never needed for correctness: every tile meets the same accuracy bound):
 *   SYMT_GEMM_TILE=<name>  restricts the sector product to one tile where that
 *                          tile applies (F64/F32: "128x96", "d96x96s2", ...,
 *                          "rows" = the row-streaming product taken by default
 *                          where K and N are at most 64 and the slices hold at
 *                          least 16384 rows in all, "tallk" = the long-K
 *                          product taken by default where M and N are at most
 *                          64 and K is 1024 or more;
 *                          BF16X3: "b128x128k32", "bd128x256s3", ...); an
 *                          unknown or inapplicable name is ignored.
 *   SYMT_GEMM_SK=0 | 1     0 forbids stream-K and split K (the long-K product's
 *                          ranges included); 1 forces stream-K on
 *                          the global-to-LDS tiles.
 *   SYMT_FUSED_V=0         keeps V aligned in the fused product (info.fused_v = 0).
 *   SYMT_GEMM_GROUP_M=<n>  M-panels per group in the tile order of the wide
 *                          split-bf16 tiles (default 8).
 *   SYMT_BF16_IL=0         keeps the wide split-bf16 tiles' planes one after the
 *                          other (not interleaved by K-steps).
 *   SYMT_BF16_FA=0         keeps u on planes for the 256 x 256 wide split-bf16
 *                          tile (not read in place).
 */
#ifndef SYMTENSOR_H
#define SYMTENSOR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SYMT_MAX_FACTORS 4   /* cyclic factors of G */
#define SYMT_MAX_ORDER 12    /* modes per operand */

enum {
  SYMT_OK = 0,
  SYMT_EINVAL = -1,        /* null pointer, negative or mismatched sizes, bad group */
  SYMT_EEINSUM = -2,       /* malformed subscripts, an empty term (s = t = 0), repeated letter
                              in a term, a letter in all three terms or in only one */
  SYMT_ESYM = -3,          /* mixed sign ratio over contracted modes, W's rule differs from the
                              derived one, bad sign string or charge */
  SYMT_EDTYPE = -4,        /* unsupported storage dtype / compute mode pair */
  SYMT_EWORKSPACE = -5,    /* workspace or aligned buffer too small */
  SYMT_EALIAS = -6,        /* output overlaps an input */
  SYMT_EUNSUPPORTED = -7,  /* valid request outside this library's support */
  SYMT_EHIP = -8           /* HIP runtime error (launch, device query) */
};

/* Complex dtypes hold (re, im) pairs, interleaved; see COMPLEX OPERANDS. */
typedef enum { SYMT_F64 = 0, SYMT_F32 = 1, SYMT_C128 = 2, SYMT_C64 = 3 } symt_dtype;
typedef enum {
  SYMT_COMPUTE_F64 = 0,    /* binary64 MFMA products */
  SYMT_COMPUTE_F32 = 1,    /* binary32 MFMA products, binary32 accumulation */
  SYMT_COMPUTE_BF16X3 = 2  /* split-bfloat16 three-term products (see above) */
} symt_compute;

/* OR-ed into a compute argument of symtensor_plan / workspace_size / contract:
 * run the three separate steps (align U, align V, product, unalign W) even
 * where the fused product applies (see FUSED PRODUCT). */
#define SYMT_FLAG_STEPS 0x100

/* G = Z_order[0] x ... x Z_order[nfactors-1]; 1 <= nfactors <= SYMT_MAX_FACTORS. */
typedef struct {
  int32_t nfactors;
  int32_t order[SYMT_MAX_FACTORS];
} symt_group;

/* One operand.  `signs` holds nmodes characters '+' / '-' (c_m, einsum-term
 * order); `charge` is Z in [0,|G|); `dims` holds the nmodes block sizes n_m
 * (each >= 0); `data` is a device pointer to the standard reduced form in
 * `dtype`, or NULL when the tensor has no elements or is only being planned.
 *
 * `mode_charges` (host pointer, may be NULL) relabels sectors: row m (|G|
 * int32) gives the charge carried by each sector label of mode m, a
 * permutation of 0..|G|-1, and the rule of Eq. symtsr reads
 * sum_m c_m chi_m(I_m) == Z.  NULL means every label is its own charge.
 * Reduced forms stay indexed by label.  A contracted mode must carry the same
 * row in u and v, and w's rows must be the derived ones (u's on I modes, v's
 * on J modes; NULL stands for identity rows) -- else SYMT_ESYM; a row that is
 * not a permutation is SYMT_EINVAL.  Supported by symtensor_plan and
 * symtensor_contract; symtensor_align and symtensor_unalign return
 * SYMT_EUNSUPPORTED for non-identity tables (their device copies live in the
 * contraction's workspace).
 *
 * `sectors` (host pointer, may be NULL) gives each mode's number of sectors
 * H_m, a divisor of |G| (Sec. 2.2, Eq. symtsr): mode m then carries the
 * coefficient c_m = sign_m |G| / H_m and sectors 0..H_m-1, and the standard
 * reduced form is [H_0]..[H_{N-2}] + dims.  NULL means |G| for every mode.
 * Stored sector tuples whose last sector has no solution hold no block (their
 * entries are ignored on input and written as zero on output).  A contracted
 * mode needs the same count in u and v, w's counts must be the derived ones
 * (u's on I modes, v's on J modes) -- else SYMT_ESYM; a count that does not
 * divide |G| is SYMT_EINVAL.  Counts below |G| need a cyclic group and no
 * charge tables (SYMT_EUNSUPPORTED), and disable the fused product. */
typedef struct {
  int32_t nmodes;
  const char* signs;
  int32_t charge;
  const int64_t* dims;
  int32_t dtype;           /* symt_dtype */
  void* data;
  const int32_t* mode_charges;
  const int32_t* sectors;
} symt_tensor;

/* Result of planning one contraction (host-only, no device needed). */
typedef struct {
  int32_t s, t, v;                 /* modes of I, J, K */
  int32_t sigma;                   /* c^V_k / c^U_k */
  int32_t group_size;              /* |G| = batch of the aligned product */
  int64_t m, k, n;                 /* aligned product shape per Q (the real product for complex) */
  int64_t elems_u, elems_v, elems_w;
  double flops;                    /* 2 |G| m k n (2 m k n with Q pinned): allowed blocks only */
  size_t bytes_u_al, bytes_v_al, bytes_w_al;  /* whole aligned forms (all |G| slices) in this
                                                 compute mode's layout */
  size_t workspace_bytes;          /* what symtensor_contract needs */
  char w_signs[SYMT_MAX_ORDER + 1];/* derived output sign string (tw order), NUL-terminated */
  int32_t w_charge;                /* derived output charge */
  int32_t fused;                   /* 1 if symtensor_contract's product reads u in place (and
                                      writes w in place): see FUSED PRODUCT */
  int32_t fused_v;                 /* 1 if the product also reads v in place (no V_al), given
                                      16-byte aligned v data */
  int32_t fused_w;                 /* 1 if the product writes w in place (fused = 1, or u
                                      aligned first: see FUSED PRODUCT) */
} symt_plan_info;

typedef struct symt_ctx symt_ctx;

/* Create a context bound to HIP device `device` (it becomes current on the
 * calling thread).  *out receives the context; SYMT_EHIP if the device does
 * not exist. */
int symtensor_create(symt_ctx** out, int device);

/* Destroy a context; NULL is a no-op.  Does not synchronise any stream. */
int symtensor_destroy(symt_ctx* ctx);

/* Validate a contraction and report its shapes, flops, derived output rule and
 * workspace size (Alg. 2, coefficient and delta steps).  Host-only: operand
 * `data` pointers are not read.  `w` may be NULL, in which case only the
 * derived rule is reported.  `compute` is a symt_compute. */
int symtensor_plan(const char* einsum, const symt_group* group, const symt_tensor* u,
                   const symt_tensor* v, const symt_tensor* w, int32_t compute,
                   symt_plan_info* info);

/* Workspace bytes needed by symtensor_contract (same as info.workspace_bytes). */
int symtensor_workspace_size(const char* einsum, const symt_group* group, const symt_tensor* u,
                             const symt_tensor* v, const symt_tensor* w, int32_t compute,
                             size_t* bytes);

/* W = contraction of U and V (Eq. ctr), written over w->data in W's standard
 * reduced form: steps (a), (b), (c) above, enqueued on `stream`.  `workspace`
 * is a caller-owned, 16-byte aligned device buffer of at least
 * info.workspace_bytes bytes holding U_al, V_al and W_al (256-byte aligned
 * sub-buffers, in that order), or for the fused product V_al and the offset
 * tables; then, where the product runs stream-K (see symtensor_sector_gemm),
 * the pieces of the tiles it cuts; then, with non-identity charge tables,
 * their device copies.  With BF16X3 the workspace's U_al and V_al planes hold
 * K at a pitch rounded up to a multiple of 8 (the pad cleared to zero), so
 * any contracted extent works; the standalone symtensor_align layouts keep K
 * unpadded.
 * w->data must not overlap u->data, v->data or the workspace, and u->data and
 * v->data must not overlap the workspace (SYMT_EALIAS).
 * Storage dtypes: SYMT_COMPUTE_F64 takes any mix of F64/F32 operands
 * (converted exactly to binary64); SYMT_COMPUTE_F32 and BF16X3 take any mix,
 * F64 inputs being rounded to binary32 first.  Complex operands likewise mix
 * C128 and C64 under F64 and F32 (see COMPLEX OPERANDS). */
int symtensor_contract(symt_ctx* ctx, const char* einsum, const symt_group* group,
                       const symt_tensor* u, const symt_tensor* v, const symt_tensor* w,
                       int32_t compute, void* workspace, size_t workspace_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * contraction as symtensor_contract, with the same arguments, results and
 * errors, but no workspace argument.  Its workspace is a device array of
 * SYMT_STATIC_WORKSPACE_BYTES that the library keeps on every device it runs
 * on (its address is resolved by symtensor_create for the context's device;
 * the array lives until the process ends).  The call allocates nothing (no
 * hipMalloc, no HIP event: symtensor_set_timing records nothing for it).
 * Where the plan's stream-K pieces would not fit, the product runs one
 * workgroup per tile instead (the results then differ from
 * symtensor_contract's in summation order only, within the same bound); a
 * contraction whose workspace still exceeds the array (large aligned forms)
 * returns SYMT_EWORKSPACE before any launch.  Every call on a device shares
 * that device's array, which keeps the last call's contents: calls that
 * overlap on one device (several streams or threads) race on it and must be
 * ordered by the caller.  u->data and v->data must not lie in the array. */
#define SYMT_STATIC_WORKSPACE_BYTES ((size_t)128 << 20)
int symtensor_contract_static(symt_ctx* ctx, const char* einsum, const symt_group* group,
                              const symt_tensor* u, const symt_tensor* v, const symt_tensor* w,
                              int32_t compute, void* stream);

/* Step (a) alone: write the aligned form of U (operand = 0) or V (operand = 1)
 * for this contraction into the caller's device buffer `aligned`
 * (at least info.bytes_u_al / bytes_v_al bytes), in the layout of the compute
 * mode (see ALIGNED LAYOUTS).  Pure data movement for F64/F32: bit-exact. */
int symtensor_align(symt_ctx* ctx, const char* einsum, const symt_group* group,
                    const symt_tensor* u, const symt_tensor* v, const symt_tensor* w,
                    int32_t compute, int32_t operand, void* aligned, size_t aligned_bytes,
                    void* stream);

/* Step (c) alone: read the aligned output W_al (layout of the compute mode,
 * info.bytes_w_al bytes) and write W's standard reduced form to w->data. */
int symtensor_unalign(symt_ctx* ctx, const char* einsum, const symt_group* group,
                      const symt_tensor* u, const symt_tensor* v, const symt_tensor* w,
                      int32_t compute, const void* aligned_w, void* stream);

/* Step (b) alone: c[q] = a[q] b[q] for q < batch over the aligned layouts of
 * the compute mode (a: batch x m x k, b: batch x k x n, or for BF16X3 the hi/lo
 * planes with b stored batch x n x k; c: batch x m x n in f64 for F64 and
 * BF16X3, f32 for F32).  c must not overlap a, b or the workspace
 * (SYMT_EALIAS).
 * `workspace` (caller-owned device memory, 16-byte aligned, may be NULL) lets
 * an F64 / F32 product run stream-K where the launch model prefers it: a fixed
 * set of persistent workgroups takes equal shares of all tiles' K-iterations,
 * so the last wave of tiles no longer idles most of the device; tiles cut
 * between two workgroups are stored here as pieces and summed afterwards in K
 * order (the result does not depend on scheduling).  It also holds split-K
 * partial tiles and the long-K product's range partials (m, n <= 64).  With a
 * NULL or smaller workspace the product runs one workgroup per tile.  The
 * launches differ only in floating-point summation order.  BF16X3 needs k a
 * multiple of 8 here (SYMT_EUNSUPPORTED otherwise). */
int symtensor_sector_gemm(symt_ctx* ctx, int32_t compute, int64_t batch, int64_t m, int64_t k,
                          int64_t n, const void* a, const void* b, void* c, void* workspace,
                          size_t workspace_bytes, void* stream);

/* Workspace bytes with which symtensor_sector_gemm may run stream-K for this
 * shape (0: the model keeps one workgroup per tile).  Host-only. */
int symtensor_sector_gemm_workspace_size(int32_t compute, int64_t batch, int64_t m, int64_t k,
                                         int64_t n, size_t* bytes);

/* Per-step timing: when enabled, symtensor_contract records a HIP event
 * pair around each of its kernel launches on the caller's stream.
 * symtensor_read_timing synchronises on those events and returns the summed
 * milliseconds and launch counts per step: [0] align U, [1] align V,
 * [2] sector product, [3] unalign W, then clears them. */
int symtensor_set_timing(symt_ctx* ctx, int32_t enable);
int symtensor_read_timing(symt_ctx* ctx, double ms[4], int64_t launches[4]);

/* Static description of a status code. */
const char* symtensor_status_string(int status);

/* Detail of the last failure on this context ("" if none); valid until the
 * next call on the context.  NULL ctx -> the detail of the last failure of a
 * context-free call (symtensor_plan, symtensor_workspace_size) on this thread. */
const char* symtensor_last_error(const symt_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* SYMTENSOR_H */

// C ABI of the irrep-alignment contraction: contexts, validation, workspace
// layout and the three-step launch sequence (align U, align V, sector
// product, unalign W).  Declarations and contracts are in include/symtensor.h.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "plan.hpp"
#include "symtensor.h"

namespace symt {
int launch_xform(const XformParams& p, bool in_f64, int out, const void* src, void* dst,
                 hipStream_t stream, std::string* err);
int launch_sector_gemm(int compute, int64_t batch, int64_t m, int64_t k, int64_t n, const void* A,
                       const void* B, void* C, hipStream_t stream, std::string* err,
                       const FusedTables* fused = nullptr, void* part = nullptr,
                       size_t part_bytes = 0, int64_t plane_a = 0, int64_t plane_b = 0, bool il = false);
int launch_offsets(const OffsetBatch& batch, hipStream_t stream, std::string* err);
int launch_put_i32(int32_t* dst, const int32_t* src, int64_t n, hipStream_t stream, std::string* err);
int launch_zero(void* ptr, size_t bytes, hipStream_t stream, std::string* err);
int launch_cplx_rows(void* v, bool f64, int64_t slices, int64_t rows, int64_t pairs, hipStream_t stream,
                     std::string* err);
int launch_cplx_rows_planes(void* v, int64_t plane, int64_t slices, int64_t rows, int64_t pairs, int64_t kp,
                            hipStream_t stream, std::string* err);
int scratch_setup(int device, std::string* err);
void* scratch_device_ptr(int device);
}  // namespace symt

using symt::Plan;

// Device copies of one plan's offset tables (the fused product's separable
// row / column offsets).  They depend on the plan only, so the context builds
// them once, on the stream of the first call that needs them, and later calls
// wait for that build (an event) instead of rebuilding.
struct TableCache {
  std::mutex mu;
  void* dev = nullptr;
  size_t bytes = 0;
  hipEvent_t ready = nullptr;
  bool built = false;
  bool done = false;       // the build has completed: no wait needed
  bool refused = false;    // no device memory (or over the context's budget): use the workspace
  ~TableCache() {
    if (ready) (void)hipEventDestroy(ready);
    if (dev) (void)hipFree(dev);
  }
};

struct CachedPlan {
  Plan plan;
  std::shared_ptr<TableCache> tables;
};

struct symt_ctx {
  int device = 0;
  std::string last_error;
  bool timing = false;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[4];
  // Plans of contractions already validated on this context, keyed by every
  // planning input except the data pointers (see plan_key), with their tables.
  std::mutex plan_mu;
  std::unordered_map<std::string, CachedPlan> plans;
  size_t table_bytes = 0;  // device bytes held by cached tables (under plan_mu)
};

namespace {

thread_local std::string g_free_error;

int ctx_fail(symt_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->last_error = msg;
  else g_free_error = msg;
  return code;
}

size_t elem_bytes(int dtype) { return dtype == SYMT_C128 ? 16 : dtype == SYMT_F64 || dtype == SYMT_C64 ? 8 : 4; }

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  if (!a || !b || na == 0 || nb == 0) return false;
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + nb && y < x + na;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

hipEvent_t take_event(symt_ctx* ctx) {
  if (!ctx->pool.empty()) {
    hipEvent_t e = ctx->pool.back();
    ctx->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Runs `fn` on the stream, bracketed by a timing event pair when timing is on.
template <typename F>
int timed(symt_ctx* ctx, int step, hipStream_t s, F&& fn) {
  hipEvent_t a = nullptr, b = nullptr;
  if (ctx->timing) {
    a = take_event(ctx);
    b = take_event(ctx);
    if (a && b) (void)hipEventRecord(a, s);
  }
  const int rc = fn();
  if (a && b) {
    (void)hipEventRecord(b, s);
    ctx->pending[step].emplace_back(a, b);
  }
  return rc;
}

int out_kind_aligned(int compute) {
  return compute == SYMT_COMPUTE_F64 ? 0 : compute == SYMT_COMPUTE_F32 ? 1 : 2;
}
int aligned_elem_bytes(int compute) {
  return compute == SYMT_COMPUTE_F64 ? 8 : compute == SYMT_COMPUTE_F32 ? 4 : 2;
}

// Align operand 0 (U) or 1 (V) from its standard form into `dst`; `chg`: the
// operand's device charge tables (nullptr: identity).
// `slice_only`: dst is the contraction's workspace copy (one slice when Q is pinned).
int do_align(symt_ctx* ctx, const Plan& p, int operand, void* dst, hipStream_t s, bool slice_only,
             const int32_t* chg = nullptr) {
  const symt::OperandDesc& X = operand == 0 ? p.U : p.V;
  if (X.elems == 0) return SYMT_OK;
  const int kind = out_kind_aligned(p.compute);
  symt::XformParams x = symt::make_xform(p, operand, true, symt::real_bytes(X.dtype),
                                         aligned_elem_bytes(p.compute), kind == 2, slice_only);
  x.chg = chg;
  if (!aligned16(X.data) || !aligned16(dst)) x.vec = 1;
  std::string err;
  const int rc = timed(ctx, operand, s, [&] {
    int r = symt::launch_xform(x, symt::real_bytes(X.dtype) == 8, kind, X.data, dst, s, &err);
    if (r == SYMT_OK && p.cplx && operand == 1) {
      // complex V: the odd real rows of the real representation of C
      const int64_t slices = slice_only ? p.nq : p.g.size;
      if (p.compute == SYMT_COMPUTE_BF16X3)
        r = symt::launch_cplx_rows_planes(dst, x.plane, slices, p.Kd, p.N, slice_only ? p.kpad : p.gk, s, &err);
      else
        r = symt::launch_cplx_rows(dst, p.compute == SYMT_COMPUTE_F64, slices, p.Kd, p.N, s, &err);
    }
    return r;
  });
  return rc ? ctx_fail(ctx, rc, err) : SYMT_OK;
}

int do_unalign(symt_ctx* ctx, const Plan& p, const void* wal, hipStream_t s, bool slice_only,
               const int32_t* chg = nullptr) {
  if (p.W.elems == 0) return SYMT_OK;
  const bool in_f64 = p.compute != SYMT_COMPUTE_F32;
  symt::XformParams x = symt::make_xform(p, 2, false, in_f64 ? 8 : 4, symt::real_bytes(p.W.dtype), false,
                                         slice_only);
  x.chg = chg;
  if (!aligned16(wal) || !aligned16(p.W.data)) x.vec = 1;
  std::string err;
  const int rc = timed(ctx, 3, s, [&] {
    // Skipped slices (s, t or v = 0, subgroup modes) leave blocks of W that no
    // product reaches, and subgroup modes stored tuples without a block: zeros.
    if (p.nq < p.g.size || p.subgroups) {
      const int r = symt::launch_zero(p.W.data, static_cast<size_t>(p.W.elems) * elem_bytes(p.W.dtype), s, &err);
      if (r) return r;
    }
    return symt::launch_xform(x, in_f64, symt::real_bytes(p.W.dtype) == 8 ? 0 : 1, wal, p.W.data, s, &err);
  });
  return rc ? ctx_fail(ctx, rc, err) : SYMT_OK;
}

// Split-bf16 planes with K padded to a multiple of 8 (kpad): clear them before
// the transforms fill their first gk columns, so the pad multiplies as zero.
int clear_k_pad(symt_ctx* ctx, const Plan& p, void* ual, void* val, hipStream_t s) {
  if (p.compute != SYMT_COMPUTE_BF16X3 || p.kpad == p.gk) return SYMT_OK;
  std::string err;
  int rc = SYMT_OK;
  if (ual && p.ws_u_al > 0) rc = symt::launch_zero(ual, p.ws_u_al, s, &err);
  if (rc == SYMT_OK && val && p.ws_v_al > 0) rc = symt::launch_zero(val, p.ws_v_al, s, &err);
  return rc ? ctx_fail(ctx, rc, err) : SYMT_OK;
}

int do_gemm(symt_ctx* ctx, int compute, int64_t batch, int64_t m, int64_t k, int64_t n,
            const void* a, const void* b, void* c, hipStream_t s,
            const symt::FusedTables* fused = nullptr, void* part = nullptr, size_t part_bytes = 0,
            int64_t plane_a = 0, int64_t plane_b = 0, bool il = false) {
  std::string err;
  const int rc = timed(ctx, 2, s, [&] {
    return symt::launch_sector_gemm(compute, batch, m, k, n, a, b, c, s, &err, fused, part, part_bytes,
                                    plane_a, plane_b, il);
  });
  return rc ? ctx_fail(ctx, rc, err) : SYMT_OK;
}

// Fused path: offset tables of U's rows and columns and of W's rows and
// columns, V aligned, then one product that reads U and writes W in place.
constexpr size_t kTableBudget = size_t(1) << 30;   // device bytes of cached tables per context

// The cached tables of `tc` (built now on `s` when `build` comes back true), or
// nullptr when the workspace must hold them: no cache slot, a captured stream
// (no allocation or cross-stream wait there), or no device memory for them.
// Called with tc->mu held.
void* cached_tables(symt_ctx* ctx, TableCache* tc, size_t bytes, hipStream_t s, bool* build) {
  *build = false;
  if (!tc || bytes == 0) return nullptr;
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess || st != hipStreamCaptureStatusNone) {
    (void)hipGetLastError();
    return nullptr;
  }
  if (!tc->dev && !tc->refused) {
    bool room;
    {
      std::lock_guard<std::mutex> lock(ctx->plan_mu);
      room = ctx->table_bytes + bytes <= kTableBudget;
      if (room) ctx->table_bytes += bytes;
    }
    if (!room || hipMalloc(&tc->dev, bytes) != hipSuccess ||
        hipEventCreateWithFlags(&tc->ready, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      if (tc->dev) (void)hipFree(tc->dev);
      tc->dev = nullptr;
      tc->refused = true;
      return nullptr;
    }
    tc->bytes = bytes;
  }
  if (!tc->dev || tc->bytes != bytes) return nullptr;
  if (!tc->built) {
    *build = true;
  } else if (!tc->done) {
    if (hipEventQuery(tc->ready) == hipSuccess) tc->done = true;
    else if (hipStreamWaitEvent(s, tc->ready, 0) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  return tc->dev;
}

int do_fused(symt_ctx* ctx, const Plan& p, char* base, hipStream_t s, const int32_t* const chg[3],
             TableCache* tc = nullptr) {
  using symt::round_up;
  const size_t G = static_cast<size_t>(p.g.size);
  // U aligned first (fused_ua): U_al, then the regions of the fused product
  void* ual = base;
  if (p.fused_ua) base += round_up(p.ws_u_al, 256);
  void* val = base;
  int64_t* ra = reinterpret_cast<int64_t*>(base + round_up(p.ws_v_al, 256));
  int64_t* ca = reinterpret_cast<int64_t*>(reinterpret_cast<char*>(ra) + round_up(8 * G * p.M, 256));
  int64_t* rc = reinterpret_cast<int64_t*>(reinterpret_cast<char*>(ca) + round_up(8 * G * p.gk, 256));
  int64_t* cc = reinterpret_cast<int64_t*>(reinterpret_cast<char*>(rc) + round_up(8 * G * p.M, 256));
  int64_t* rb = reinterpret_cast<int64_t*>(reinterpret_cast<char*>(cc) + round_up(8 * G * p.gn, 256));
  int64_t* cb = reinterpret_cast<int64_t*>(reinterpret_cast<char*>(rb) + round_up(8 * G * p.gk, 256));
  char* part = p.fused_b ? reinterpret_cast<char*>(cb) + round_up(8 * G * p.gn, 256)
                         : reinterpret_cast<char*>(rb);
  // 16-byte loads of A need every row's K run to start 16-byte aligned
  // (K stepped run by run: a run of whole vectors keeps every step's valid part whole;
  // U_al: one run of gk per row, 256-byte aligned)
  const int64_t run = p.fused_ua ? p.gk : (p.cplx ? 2 : 1) * p.nK, vw = p.compute == SYMT_COMPUTE_F64 ? 2 : 4;
  int vec = (p.fused_ua || aligned16(p.U.data)) && (p.compute == SYMT_COMPUTE_BF16X3 || run % vw == 0) ? 2 : 1;
  // K-major A: 16-byte loads along U's output modes
  if (p.a_trans) vec = aligned16(p.U.data) && p.a_chunks ? 2 : 1;
  // V in place: its column chunks take 16-byte loads (global-to-LDS tiles, and
  // register tiles whose loads are vectors), so V must be 16-byte aligned
  const bool fb = p.fused_b && (p.krun > 0 || aligned16(p.V.data));
  // vector loads of B in place need 16-byte aligned, whole column chunks
  if (fb && vec > 1 && !(aligned16(p.V.data) && p.fused_b_chunks)) vec = 1;
  std::string err;
  // the tables: cached on the context (all of the plan's tables, built once), or
  // in the workspace (the ones this call reads, built every call)
  const int n_plan = p.fused_b ? 6 : 4;
  char* const t0 = reinterpret_cast<char*>(ra);
  const size_t plan_bytes = static_cast<size_t>((p.fused_b ? reinterpret_cast<char*>(cb) +
                                                                 round_up(8 * G * p.gn, 256)
                                                           : reinterpret_cast<char*>(rb)) - t0);
  bool build = true;
  int n_build = fb ? 6 : 4;
  std::unique_lock<std::mutex> tlock;
  if (tc) tlock = std::unique_lock<std::mutex>(tc->mu);
  if (char* cached = static_cast<char*>(cached_tables(ctx, tc, plan_bytes, s, &build))) {
    auto move = [&](int64_t*& x) { x = reinterpret_cast<int64_t*>(cached + (reinterpret_cast<char*>(x) - t0)); };
    move(ra); move(ca); move(rc); move(cc); move(rb); move(cb);
    n_build = n_plan;
  } else {
    build = true;
  }
  int rc_ = SYMT_OK;
  if (build) {
    rc_ = timed(ctx, 0, s, [&] {
      symt::OffsetBatch b;
      const int ops[6] = {0, 0, 2, 2, 1, 1};
      int64_t* outs[6] = {ra, ca, rc, cc, rb, cb};
      int64_t total = 0;
      b.n = n_build;
      for (int t = 0; t < b.n; ++t) {
        if (p.fused_ua && ops[t] == 0 && !p.bf16_wide_fa)   // U_al: row m at (q M + m) gk, column k at k
          b.t[t] = t == 0 ? symt::affine_offsets(p, p.M, p.M * p.gk, p.gk) : symt::affine_offsets(p, p.gk, 0, 1);
        else
          b.t[t] = symt::make_offsets(p, ops[t], t % 2 == 0);
        b.t[t].chg = chg[ops[t]];
        b.out[t] = outs[t];
        total += b.t[t].count * G;
        b.end[t] = total;
      }
      return symt::launch_offsets(b, s, &err);
    });
    if (rc_ == SYMT_OK && tc && tc->dev && reinterpret_cast<char*>(ra) != t0 && !tc->built) {
      if (hipEventRecord(tc->ready, s) == hipSuccess) tc->built = true;
      else (void)hipGetLastError();
    }
  }
  if (tlock.owns_lock()) tlock.unlock();
  if (rc_) return ctx_fail(ctx, rc_, err);
  // split-bf16 on the 256 x 256 wide tile: binary32 U read in place (16-byte aligned)
  const bool wide_fa = p.bf16_wide_fa && aligned16(p.U.data);
  if (p.fused_ua && (rc_ = clear_k_pad(ctx, p, ual, fb ? nullptr : val, s))) return rc_;
  if (p.fused_ua && !wide_fa && (rc_ = do_align(ctx, p, 0, ual, s, true, chg[0]))) return rc_;
  if (!fb && (rc_ = do_align(ctx, p, 1, val, s, true, chg[1]))) return rc_;
  symt::FusedTables f{ra, ca, rc, cc, vec};
  // split-bf16 on aligned U: A and B come from the hi/lo planes, only W's tables apply
  if (p.fused_ua && p.compute == SYMT_COMPUTE_BF16X3 && !wide_fa) f.ra = f.ca = nullptr;
  f.a_bytes = static_cast<int32_t>(p.fused_ua && !wide_fa ? (p.compute == SYMT_COMPUTE_F64 ? 8 : 4)
                                                            : elem_bytes(p.U.dtype));
  f.krun = p.krun;
  f.at = p.a_trans ? 1 : 0;
  f.c_bytes = static_cast<int32_t>(elem_bytes(p.W.dtype));
  // W written in place with its rows contiguous (and not its columns): the
  // row-streaming product stores lanes along rows
  f.c_trans = !p.cplx && p.w_row_run >= 16 && p.w_col_run < 8 ? 1 : 0;
  // U's K index contiguous (U_al, or runs of 16 and more in U): the long-K
  // product loads A along K
  f.a_klanes = p.fused_ua || p.u_k_run >= 16 ? 1 : 0;
  f.k_groups = symt::tallk_groups(p) ? 1 : 0;
  // W's rows contiguous in runs of 4k elements: binary32 tiles store 4 rows per lane
  f.c_rows4 = !p.cplx && p.w_row_run % 4 == 0 ? 1 : 0;
  // K-major A without M chunks: 16-byte loads along U's trailing contracted run instead
  // A not K-major, its K runs whole 16-byte vectors (whatever B's layout)
  // (K stepped run by run is the register tiles' concern; the row-streaming
  // product reads each K index through its own table entry)
  f.a_krow = !p.a_trans && !p.cplx && (p.fused_ua || aligned16(p.U.data)) && run % vw == 0 ? 1 : 0;
  f.a_kvec = p.a_trans && !p.cplx && !p.a_chunks && aligned16(p.U.data) && p.u_k_run % vw == 0 &&
                     (!fb || (aligned16(p.V.data) && p.fused_b_chunks))
                 ? 1
                 : 0;
  if (fb) {
    f.rb = rb;
    f.cb = cb;
    f.ldb = p.ldb;
  }
  return do_gemm(ctx, p.compute, p.g.size, p.M, p.fused_ua ? p.kpad : p.gk, p.gn,
                 p.fused_ua && !wide_fa ? ual : p.U.data,
                 fb ? p.V.data : val,
                 p.W.data, s, &f,
                 p.bytes_partial ? part : nullptr, p.bytes_partial, 0, 0, p.bf16_il);
}

// Cache key of a planning request: the einsum, group, compute mode, every
// descriptor field but `data`, and the tuning variables the planner reads.  An
// empty key (malformed descriptors, which make_plan rejects) bypasses the cache.
constexpr size_t kMaxCachedPlans = 1024;

void key_add(std::string& k, const void* p, size_t n) { k.append(static_cast<const char*>(p), n); }

bool key_tensor(std::string& k, const symt_tensor* t, int G) {
  if (!t) {
    k.push_back('N');
    return true;
  }
  if (t->nmodes < 1 || t->nmodes > SYMT_MAX_ORDER || !t->signs || !t->dims) return false;
  const size_t n = static_cast<size_t>(t->nmodes);
  const size_t ns = strnlen(t->signs, n + 1);
  k.push_back('T');
  key_add(k, &t->nmodes, sizeof t->nmodes);
  key_add(k, &ns, sizeof ns);
  k.append(t->signs, ns);
  key_add(k, &t->charge, sizeof t->charge);
  key_add(k, &t->dtype, sizeof t->dtype);
  key_add(k, t->dims, n * sizeof(int64_t));
  k.push_back(t->mode_charges ? 'C' : 'c');
  if (t->mode_charges) key_add(k, t->mode_charges, n * static_cast<size_t>(G) * sizeof(int32_t));
  k.push_back(t->sectors ? 'S' : 's');
  if (t->sectors) key_add(k, t->sectors, n * sizeof(int32_t));
  return true;
}

std::string plan_key(const char* einsum, const symt_group* group, const symt_tensor* u, const symt_tensor* v,
                     const symt_tensor* w, int32_t compute) {
  if (!einsum || !group || !u || !v || group->nfactors < 1 || group->nfactors > SYMT_MAX_FACTORS) return {};
  int64_t G = 1;
  for (int f = 0; f < group->nfactors; ++f) {
    if (group->order[f] < 1) return {};
    G *= group->order[f];
    if (G > (1 << 20)) return {};
  }
  std::string k(einsum);
  k.push_back('\0');
  key_add(k, &group->nfactors, sizeof group->nfactors);
  key_add(k, group->order, static_cast<size_t>(group->nfactors) * sizeof(int32_t));
  key_add(k, &compute, sizeof compute);
  if (!key_tensor(k, u, static_cast<int>(G)) || !key_tensor(k, v, static_cast<int>(G)) ||
      !key_tensor(k, w, static_cast<int>(G)))
    return {};
  for (const char* var : {"SYMT_FUSED_V", "SYMT_GEMM_TILE", "SYMT_GEMM_SK", "SYMT_BF16_IL", "SYMT_BF16_FA"}) {
    const char* val = std::getenv(var);
    k.push_back('|');
    if (val) k.append(val);
  }
  return k;
}

// `tables` (optional): the cached plan's device table slot.
int plan_for(symt_ctx* ctx, const char* einsum, const symt_group* group, const symt_tensor* u,
             const symt_tensor* v, const symt_tensor* w, int32_t compute, Plan* p,
             std::shared_ptr<TableCache>* tables = nullptr) {
  std::string key;
  if (ctx) {
    key = plan_key(einsum, group, u, v, w, compute);
    if (!key.empty()) {
      std::lock_guard<std::mutex> lock(ctx->plan_mu);
      auto it = ctx->plans.find(key);
      if (it != ctx->plans.end()) {
        *p = it->second.plan;
        p->U.data = u->data;
        p->V.data = v->data;
        p->W.data = w ? w->data : nullptr;
        if (tables) *tables = it->second.tables;
        return SYMT_OK;
      }
    }
  }
  std::string err;
  const int rc = symt::make_plan(einsum, group, u, v, w, compute, p, &err);
  if (rc) return ctx_fail(ctx, rc, err);
  if (!key.empty()) {
    std::lock_guard<std::mutex> lock(ctx->plan_mu);
    if (ctx->plans.size() >= kMaxCachedPlans) {
      // (a call still holding a plan's tables keeps them alive until it returns;
      // freeing device memory waits for the device)
      ctx->plans.clear();
      ctx->table_bytes = 0;
    }
    auto tc = std::make_shared<TableCache>();
    ctx->plans.emplace(std::move(key), CachedPlan{*p, tc});
    if (tables) *tables = tc;
  }
  return SYMT_OK;
}

int check_data(symt_ctx* ctx, const symt::OperandDesc& X, const char* name) {
  if (X.elems > 0 && !X.data)
    return ctx_fail(ctx, SYMT_EINVAL, std::string("operand ") + name + " data is NULL");
  return SYMT_OK;
}

int set_device(symt_ctx* ctx) {
  const hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return ctx_fail(ctx, SYMT_EHIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
  return SYMT_OK;
}

}  // namespace

extern "C" {

int symtensor_create(symt_ctx** out, int device) {
  if (!out) return ctx_fail(nullptr, SYMT_EINVAL, "out is NULL");
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || device < 0 || device >= count)
    return ctx_fail(nullptr, SYMT_EHIP, "no such HIP device");
  e = hipSetDevice(device);
  if (e != hipSuccess) return ctx_fail(nullptr, SYMT_EHIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
  // the allocation-free entry point's device array: its address on this device
  std::string err;
  const int rc = symt::scratch_setup(device, &err);
  if (rc) return ctx_fail(nullptr, rc, err);
  symt_ctx* c = new symt_ctx;
  c->device = device;
  *out = c;
  return SYMT_OK;
}

int symtensor_destroy(symt_ctx* ctx) {
  if (!ctx) return SYMT_OK;
  for (auto& v : ctx->pending)
    for (auto& pr : v) {
      hipEventDestroy(pr.first);
      hipEventDestroy(pr.second);
    }
  for (hipEvent_t e : ctx->pool) hipEventDestroy(e);
  delete ctx;
  return SYMT_OK;
}

int symtensor_plan(const char* einsum, const symt_group* group, const symt_tensor* u,
                   const symt_tensor* v, const symt_tensor* w, int32_t compute,
                   symt_plan_info* info) {
  if (!info) return ctx_fail(nullptr, SYMT_EINVAL, "info is NULL");
  Plan p;
  int rc = plan_for(nullptr, einsum, group, u, v, w, compute, &p);
  if (rc) return rc;
  std::memset(info, 0, sizeof *info);
  info->s = p.s;
  info->t = p.t;
  info->v = p.v;
  info->sigma = p.sigma;
  info->group_size = p.g.size;
  info->m = p.M;
  info->k = p.gk;
  info->n = p.gn;
  info->elems_u = p.U.elems;
  info->elems_v = p.V.elems;
  info->elems_w = p.W.elems;
  info->flops = p.flops;
  info->bytes_u_al = p.bytes_u_al;
  info->bytes_v_al = p.bytes_v_al;
  info->bytes_w_al = p.bytes_w_al;
  info->workspace_bytes = p.workspace;
  for (size_t m = 0; m < p.tw.size(); ++m) info->w_signs[m] = p.w_sign[m] > 0 ? '+' : '-';
  info->w_signs[p.tw.size()] = '\0';
  info->w_charge = p.w_charge;
  info->fused = p.fused ? 1 : 0;
  info->fused_v = p.fused_b ? 1 : 0;
  info->fused_w = (p.fused || p.fused_ua) ? 1 : 0;
  return SYMT_OK;
}

int symtensor_workspace_size(const char* einsum, const symt_group* group, const symt_tensor* u,
                             const symt_tensor* v, const symt_tensor* w, int32_t compute,
                             size_t* bytes) {
  if (!bytes) return ctx_fail(nullptr, SYMT_EINVAL, "bytes is NULL");
  Plan p;
  const int rc = plan_for(nullptr, einsum, group, u, v, w, compute, &p);
  if (rc) return rc;
  *bytes = p.workspace;
  return SYMT_OK;
}

}  // extern "C"

namespace {
// Validation and launches of one planned contraction (symtensor_contract and
// symtensor_contract_static): every check runs before the first launch.
int contract_planned(symt_ctx* ctx, const Plan& p, void* workspace, size_t workspace_bytes, void* stream,
                     TableCache* tables = nullptr) {
  int rc;
  if ((rc = check_data(ctx, p.U, "u")) || (rc = check_data(ctx, p.V, "v")) ||
      (rc = check_data(ctx, p.W, "w")))
    return rc;
  if (p.W.elems == 0) return SYMT_OK;
  if (workspace_bytes < p.workspace || (p.workspace > 0 && !workspace))
    return ctx_fail(ctx, SYMT_EWORKSPACE, "workspace smaller than symtensor_workspace_size()");
  const size_t wb = static_cast<size_t>(p.W.elems) * elem_bytes(p.W.dtype);
  const size_t ub = static_cast<size_t>(p.U.elems) * elem_bytes(p.U.dtype),
               vb = static_cast<size_t>(p.V.elems) * elem_bytes(p.V.dtype);
  if (overlaps(p.W.data, wb, p.U.data, ub) || overlaps(p.W.data, wb, p.V.data, vb) ||
      overlaps(p.W.data, wb, workspace, p.workspace))
    return ctx_fail(ctx, SYMT_EALIAS, "output overlaps an input or the workspace");
  // the workspace is written (aligned forms, tables, pieces) before u and v are read
  if (overlaps(p.U.data, ub, workspace, p.workspace) || overlaps(p.V.data, vb, workspace, p.workspace))
    return ctx_fail(ctx, SYMT_EALIAS, "an input overlaps the workspace");
  if (p.workspace > 0 && !aligned16(workspace))
    return ctx_fail(ctx, SYMT_EUNSUPPORTED, "workspace must be 16-byte aligned");
  if ((rc = set_device(ctx))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(workspace);
  // charge tables: forward and inverse per mode, uploaded into the workspace's last region
  const int32_t* chg[3] = {nullptr, nullptr, nullptr};
  if (p.charges) {
    int32_t* dev = reinterpret_cast<int32_t*>(base + p.workspace - symt::round_up(p.bytes_charges, 256));
    int64_t off[3];
    const std::vector<int32_t> host = symt::charge_tables_device(p, off);
    std::string err;
    if ((rc = symt::launch_put_i32(dev, host.data(), static_cast<int64_t>(host.size()), s, &err)))
      return ctx_fail(ctx, rc, err);
    for (int op = 0; op < 3; ++op)
      if (!p.chg[op].empty()) chg[op] = dev + off[op];
  }
  if (p.fused || p.fused_ua) return do_fused(ctx, p, base, s, chg, tables);
  void* ual = base;
  void* val = base + symt::round_up(p.ws_u_al, 256);
  void* wal = base + symt::round_up(p.ws_u_al, 256) + symt::round_up(p.ws_v_al, 256);
  char* part = static_cast<char*>(wal) + symt::round_up(p.ws_w_al, 256);
  if ((rc = clear_k_pad(ctx, p, ual, val, s))) return rc;
  if ((rc = do_align(ctx, p, 0, ual, s, true, chg[0]))) return rc;
  if ((rc = do_align(ctx, p, 1, val, s, true, chg[1]))) return rc;
  // the workspace holds the nq live slices in order: one batched product of them
  // (none live: no block of W is reached, and the unalign step clears W)
  if (p.nq > 0 && (rc = do_gemm(ctx, p.compute, p.nq, p.M, p.kpad, p.gn, ual, val, wal, s, nullptr,
                                p.bytes_partial ? part : nullptr, p.bytes_partial, 0, 0, p.bf16_il)))
    return rc;
  if ((rc = do_unalign(ctx, p, wal, s, true, chg[2]))) return rc;
  return SYMT_OK;
}
}  // namespace

extern "C" {

int symtensor_contract(symt_ctx* ctx, const char* einsum, const symt_group* group,
                       const symt_tensor* u, const symt_tensor* v, const symt_tensor* w,
                       int32_t compute, void* workspace, size_t workspace_bytes, void* stream) {
  if (!ctx) return ctx_fail(nullptr, SYMT_EINVAL, "context is NULL");
  if (!w) return ctx_fail(ctx, SYMT_EINVAL, "output descriptor is NULL");
  Plan p;
  std::shared_ptr<TableCache> tables;
  int rc = plan_for(ctx, einsum, group, u, v, w, compute, &p, &tables);
  if (rc) return rc;
  return contract_planned(ctx, p, workspace, workspace_bytes, stream, tables.get());
}

int symtensor_contract_static(symt_ctx* ctx, const char* einsum, const symt_group* group,
                              const symt_tensor* u, const symt_tensor* v, const symt_tensor* w,
                              int32_t compute, void* stream) {
  if (!ctx) return ctx_fail(nullptr, SYMT_EINVAL, "context is NULL");
  if (!w) return ctx_fail(ctx, SYMT_EINVAL, "output descriptor is NULL");
  // the device address of the library's array on this context's device (never
  // the array's host-side name)
  void* scratch = symt::scratch_device_ptr(ctx->device);
  if (!scratch) return ctx_fail(ctx, SYMT_EHIP, "the library's device workspace is not set up on this device");
  Plan p;
  int rc = plan_for(ctx, einsum, group, u, v, w, compute, &p);
  if (rc) return rc;
  const size_t cap = SYMT_STATIC_WORKSPACE_BYTES;
  if (p.workspace > cap && p.bytes_partial > 0) {
    // without the stream-K pieces (or split-K partial tiles) the product runs
    // one workgroup per tile; the pieces sit just before the charge tables
    p.workspace -= symt::round_up(p.bytes_partial, 256);
    p.bytes_partial = 0;
  }
  if (p.workspace > cap)
    return ctx_fail(ctx, SYMT_EWORKSPACE,
                    "contraction needs " + std::to_string(p.workspace) +
                        " bytes of workspace; symtensor_contract_static holds " + std::to_string(cap));
  // no timing events: creating them could allocate
  const bool timing = ctx->timing;
  ctx->timing = false;
  rc = contract_planned(ctx, p, scratch, cap, stream);
  ctx->timing = timing;
  return rc;
}

int symtensor_align(symt_ctx* ctx, const char* einsum, const symt_group* group,
                    const symt_tensor* u, const symt_tensor* v, const symt_tensor* w,
                    int32_t compute, int32_t operand, void* aligned, size_t aligned_bytes,
                    void* stream) {
  if (!ctx) return ctx_fail(nullptr, SYMT_EINVAL, "context is NULL");
  if (operand != 0 && operand != 1) return ctx_fail(ctx, SYMT_EINVAL, "operand must be 0 (u) or 1 (v)");
  Plan p;
  int rc = plan_for(ctx, einsum, group, u, v, w, compute, &p);
  if (rc) return rc;
  if (p.charges)
    return ctx_fail(ctx, SYMT_EUNSUPPORTED,
                    "non-identity charge tables are supported by symtensor_contract only");
  const symt::OperandDesc& X = operand == 0 ? p.U : p.V;
  if ((rc = check_data(ctx, X, operand == 0 ? "u" : "v"))) return rc;
  const size_t need = operand == 0 ? p.bytes_u_al : p.bytes_v_al;
  if (aligned_bytes < need || (need > 0 && !aligned))
    return ctx_fail(ctx, SYMT_EWORKSPACE, "aligned buffer too small");
  if (overlaps(aligned, need, X.data, static_cast<size_t>(X.elems) * elem_bytes(X.dtype)))
    return ctx_fail(ctx, SYMT_EALIAS, "aligned buffer overlaps the operand");
  if ((rc = set_device(ctx))) return rc;
  if (symt::pinned_form(p, operand) && need > 0) {
    // Q pinned: the other slices of the aligned form are zero (Alg. 2's deltas)
    std::string err;
    if ((rc = symt::launch_zero(aligned, need, static_cast<hipStream_t>(stream), &err)))
      return ctx_fail(ctx, rc, err);
  }
  return do_align(ctx, p, operand, aligned, static_cast<hipStream_t>(stream), false);
}

int symtensor_unalign(symt_ctx* ctx, const char* einsum, const symt_group* group,
                      const symt_tensor* u, const symt_tensor* v, const symt_tensor* w,
                      int32_t compute, const void* aligned_w, void* stream) {
  if (!ctx) return ctx_fail(nullptr, SYMT_EINVAL, "context is NULL");
  if (!w) return ctx_fail(ctx, SYMT_EINVAL, "output descriptor is NULL");
  Plan p;
  int rc = plan_for(ctx, einsum, group, u, v, w, compute, &p);
  if (rc) return rc;
  if (p.charges)
    return ctx_fail(ctx, SYMT_EUNSUPPORTED,
                    "non-identity charge tables are supported by symtensor_contract only");
  if ((rc = check_data(ctx, p.W, "w"))) return rc;
  if (p.W.elems > 0 && !aligned_w) return ctx_fail(ctx, SYMT_EINVAL, "aligned_w is NULL");
  if (overlaps(p.W.data, static_cast<size_t>(p.W.elems) * elem_bytes(p.W.dtype), aligned_w,
               p.bytes_w_al))
    return ctx_fail(ctx, SYMT_EALIAS, "output overlaps the aligned buffer");
  if ((rc = set_device(ctx))) return rc;
  return do_unalign(ctx, p, aligned_w, static_cast<hipStream_t>(stream), false);
}

int symtensor_sector_gemm_workspace_size(int32_t compute, int64_t batch, int64_t m, int64_t k,
                                         int64_t n, size_t* bytes) {
  if (!bytes) return ctx_fail(nullptr, SYMT_EINVAL, "bytes is NULL");
  *bytes = 0;
  if (compute < SYMT_COMPUTE_F64 || compute > SYMT_COMPUTE_BF16X3)
    return ctx_fail(nullptr, SYMT_EDTYPE, "unknown compute mode");
  if (batch < 0 || m < 0 || k < 0 || n < 0) return ctx_fail(nullptr, SYMT_EINVAL, "negative size");
  if (compute != SYMT_COMPUTE_BF16X3 && batch > 0 && m > 0 && k > 0 && n > 0)
    *bytes = symt::choose_fp_gemm(batch, m, n, k, compute == SYMT_COMPUTE_F64 ? 8 : 4, true).partial_bytes;
  return SYMT_OK;
}

int symtensor_sector_gemm(symt_ctx* ctx, int32_t compute, int64_t batch, int64_t m, int64_t k,
                          int64_t n, const void* a, const void* b, void* c, void* workspace,
                          size_t workspace_bytes, void* stream) {
  if (!ctx) return ctx_fail(nullptr, SYMT_EINVAL, "context is NULL");
  if (compute < SYMT_COMPUTE_F64 || compute > SYMT_COMPUTE_BF16X3)
    return ctx_fail(ctx, SYMT_EDTYPE, "unknown compute mode");
  if (batch < 0 || m < 0 || k < 0 || n < 0) return ctx_fail(ctx, SYMT_EINVAL, "negative size");
  const size_t ea = compute == SYMT_COMPUTE_F64 ? 8 : compute == SYMT_COMPUTE_F32 ? 4 : 4;
  const size_t ec = compute == SYMT_COMPUTE_F32 ? 4 : 8;
  const size_t na = static_cast<size_t>(batch) * m * k * ea, nb = static_cast<size_t>(batch) * k * n * ea,
               nc = static_cast<size_t>(batch) * m * n * ec;
  if (nc == 0) return SYMT_OK;
  if (!c || (na && !a) || (nb && !b)) return ctx_fail(ctx, SYMT_EINVAL, "NULL buffer");
  if (overlaps(c, nc, a, na) || overlaps(c, nc, b, nb))
    return ctx_fail(ctx, SYMT_EALIAS, "c overlaps a or b");
  if (compute == SYMT_COMPUTE_BF16X3 && (k % 8 != 0 || !aligned16(a) || !aligned16(b)))
    return ctx_fail(ctx, SYMT_EUNSUPPORTED, "split-bf16 product needs k % 8 == 0 and 16-byte aligned planes");
  if (compute != SYMT_COMPUTE_BF16X3 && (!aligned16(a) || !aligned16(b) || !aligned16(c)))
    return ctx_fail(ctx, SYMT_EUNSUPPORTED, "sector product buffers must be 16-byte aligned");
  if (!workspace) workspace_bytes = 0;
  if (workspace_bytes && !aligned16(workspace))
    return ctx_fail(ctx, SYMT_EUNSUPPORTED, "workspace must be 16-byte aligned");
  if (overlaps(c, nc, workspace, workspace_bytes) || overlaps(a, na, workspace, workspace_bytes) ||
      overlaps(b, nb, workspace, workspace_bytes))
    return ctx_fail(ctx, SYMT_EALIAS, "workspace overlaps a, b or c");
  int rc = set_device(ctx);
  if (rc) return rc;
  return do_gemm(ctx, compute, batch, m, k, n, a, b, c, static_cast<hipStream_t>(stream), nullptr,
                 workspace_bytes ? workspace : nullptr, workspace_bytes);
}

int symtensor_set_timing(symt_ctx* ctx, int32_t enable) {
  if (!ctx) return ctx_fail(nullptr, SYMT_EINVAL, "context is NULL");
  ctx->timing = enable != 0;
  return SYMT_OK;
}

int symtensor_read_timing(symt_ctx* ctx, double ms[4], int64_t launches[4]) {
  if (!ctx || !ms || !launches) return ctx_fail(ctx, SYMT_EINVAL, "NULL argument");
  for (int i = 0; i < 4; ++i) {
    ms[i] = 0.0;
    launches[i] = 0;
    for (auto& pr : ctx->pending[i]) {
      float t = 0.f;
      if (hipEventSynchronize(pr.second) == hipSuccess &&
          hipEventElapsedTime(&t, pr.first, pr.second) == hipSuccess) {
        ms[i] += t;
        ++launches[i];
      }
      ctx->pool.push_back(pr.first);
      ctx->pool.push_back(pr.second);
    }
    ctx->pending[i].clear();
  }
  return SYMT_OK;
}

const char* symtensor_status_string(int status) {
  switch (status) {
    case SYMT_OK: return "ok";
    case SYMT_EINVAL: return "invalid argument";
    case SYMT_EEINSUM: return "invalid einsum subscripts";
    case SYMT_ESYM: return "inconsistent symmetry";
    case SYMT_EDTYPE: return "unsupported dtype or compute mode";
    case SYMT_EWORKSPACE: return "workspace too small";
    case SYMT_EALIAS: return "output overlaps an input";
    case SYMT_EUNSUPPORTED: return "unsupported request";
    case SYMT_EHIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char* symtensor_last_error(const symt_ctx* ctx) {
  return ctx ? ctx->last_error.c_str() : g_free_error.c_str();
}

}  // extern "C"

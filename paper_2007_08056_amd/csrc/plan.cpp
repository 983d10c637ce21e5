// Host planner: einsum parsing, mode classification, the derived output rule,
// aligned shapes and the transform descriptors (Alg. 2: its coefficient
// and delta steps, and the index maps of its aligned-operand and final steps).
#include "plan.hpp"

#include <algorithm>
#include <cstdio>
#include <climits>
#include <cstdlib>
#include <string>
#include <cstring>
#include <numeric>

namespace symt {

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

namespace {

constexpr int64_t kInt64Max = INT64_MAX;

bool mul_ok(int64_t a, int64_t b, int64_t* out) {
  if (a < 0 || b < 0) return false;
  if (a != 0 && b > kInt64Max / a) return false;
  *out = a * b;
  return true;
}

int fail(std::string* err, int code, const char* fmt, const char* a = "", const char* b = "") {
  if (err) {
    char buf[256];
    std::snprintf(buf, sizeof buf, fmt, a, b);
    *err = buf;
  }
  return code;
}

int gsub(const GroupDesc& g, int a, int b);
int gadd(const GroupDesc& g, int a, int b) {
  int r = 0, mul = 1;
  for (int f = g.nf - 1; f >= 0; --f) {
    const int o = g.ord[f];
    const int da = a % o, db = b % o;
    a /= o;
    b /= o;
    r += ((da + db) % o) * mul;
    mul *= o;
  }
  return r;
}
int gneg(const GroupDesc& g, int a) {
  int r = 0, mul = 1;
  for (int f = g.nf - 1; f >= 0; --f) {
    const int o = g.ord[f];
    const int da = a % o;
    a /= o;
    r += ((o - da) % o) * mul;
    mul *= o;
  }
  return r;
}
int gsub(const GroupDesc& g, int a, int b) { return gadd(g, a, gneg(g, b)); }
int gtimes(const GroupDesc& g, int c, int a) { return c >= 0 ? a : gneg(g, a); }

int read_group(const symt_group* grp, GroupDesc* g, std::string* err) {
  if (!grp) return fail(err, SYMT_EINVAL, "group is NULL");
  if (grp->nfactors < 1 || grp->nfactors > SYMT_MAX_FACTORS)
    return fail(err, SYMT_EINVAL, "group must have 1..%s cyclic factors", "4");
  g->nf = grp->nfactors;
  int64_t size = 1;
  for (int f = 0; f < g->nf; ++f) {
    if (grp->order[f] < 1) return fail(err, SYMT_EINVAL, "group factor orders must be >= 1");
    g->ord[f] = grp->order[f];
    size *= grp->order[f];
    if (size > (1 << 20)) return fail(err, SYMT_EUNSUPPORTED, "group order above 2^20");
  }
  for (int f = g->nf; f < SYMT_MAX_FACTORS; ++f) g->ord[f] = 1;
  g->size = static_cast<int32_t>(size);
  return SYMT_OK;
}

// Charge tables of an operand: n rows of |G| labels -> charges, each a
// permutation; an all-identity table is stored as empty.
int read_charges(const symt_tensor* t, const GroupDesc& g, std::vector<int32_t>* out, const char* name,
                 std::string* err) {
  out->clear();
  if (!t->mode_charges) return SYMT_OK;
  const int G = g.size;
  bool identity = true;
  std::vector<char> seen(static_cast<size_t>(G));
  for (int m = 0; m < t->nmodes; ++m) {
    std::fill(seen.begin(), seen.end(), 0);
    for (int l = 0; l < G; ++l) {
      const int32_t c = t->mode_charges[static_cast<size_t>(m) * G + l];
      if (c < 0 || c >= G || seen[c])
        return fail(err, SYMT_EINVAL, "operand %s: charge table of mode %s is not a permutation of the group",
                    name, std::to_string(m).c_str());
      seen[c] = 1;
      identity = identity && c == l;
    }
  }
  if (!identity) out->assign(t->mode_charges, t->mode_charges + static_cast<size_t>(t->nmodes) * G);
  return SYMT_OK;
}

int32_t table_at(const std::vector<int32_t>& tab, int G, int mode, int label) {
  return tab.empty() ? label : tab[static_cast<size_t>(mode) * G + label];
}

int read_operand(const symt_tensor* t, const GroupDesc& g, OperandDesc* o, const char* name,
                 std::string* err) {
  if (!t) return fail(err, SYMT_EINVAL, "operand %s is NULL", name);
  if (t->nmodes < 1 || t->nmodes > kMaxOrder)
    return fail(err, SYMT_EINVAL, "operand %s: order must be 1..12", name);
  if (!t->signs) return fail(err, SYMT_ESYM, "operand %s: sign string is NULL", name);
  if (!t->dims) return fail(err, SYMT_EINVAL, "operand %s: dims is NULL", name);
  o->n = t->nmodes;
  for (int m = 0; m < o->n; ++m) {
    const char c = t->signs[m];
    if (c == '+') o->sign[m] = 1;
    else if (c == '-') o->sign[m] = -1;
    else return fail(err, SYMT_ESYM, "operand %s: sign string must be '+'/'-' per mode", name);
  }
  if (t->signs[o->n] != '\0')
    return fail(err, SYMT_ESYM, "operand %s: sign string longer than its order", name);
  if (t->charge < 0 || t->charge >= g.size)
    return fail(err, SYMT_ESYM, "operand %s: charge outside [0,|G|)", name);
  o->charge = t->charge;
  if (t->dtype < SYMT_F64 || t->dtype > SYMT_C64)
    return fail(err, SYMT_EDTYPE, "operand %s: dtype must be SYMT_F64, F32, C128 or C64", name);
  o->dtype = t->dtype;
  o->data = t->data;
  for (int m = 0; m < o->n; ++m) {
    const int32_t h = t->sectors ? t->sectors[m] : g.size;
    if (h < 1 || h > g.size || g.size % h != 0)
      return fail(err, SYMT_EINVAL, "operand %s: sector count of mode %s does not divide |G|", name,
                  std::to_string(m).c_str());
    o->hs[m] = h;
  }
  int64_t e = 1;
  for (int m = 0; m < o->n - 1; ++m)
    if (!mul_ok(e, o->hs[m], &e)) return fail(err, SYMT_EINVAL, "operand %s: size overflows", name);
  for (int m = 0; m < o->n; ++m) {
    if (t->dims[m] < 0) return fail(err, SYMT_EINVAL, "operand %s: negative block dimension", name);
    o->dims[m] = t->dims[m];
    if (!mul_ok(e, t->dims[m], &e)) return fail(err, SYMT_EINVAL, "operand %s: size overflows", name);
  }
  o->elems = e;
  return SYMT_OK;
}

bool is_letter(char c) { return (c >= 'a' && c <= 'z') || (c >= 'A' && c <= 'Z'); }

}  // namespace

AlignedLayout aligned_layout(int32_t compute, int operand) {
  // The split-bf16 product reads both factors along the contracted index, so
  // V's aligned form keeps that index fastest.
  if (compute == SYMT_COMPUTE_BF16X3 && operand == 1) return kColMajor;
  return kRowMajor;
}

// The product tiles read row k0 + k of a K-step of V at rb(Q, k0) + k ldb and
// 16-byte column chunks at cb(Q, n) (single elements when K is stepped run by
// run, which needs only the first condition).  That needs, for a real V:
//  * its contracted modes, in U's K order, affine: each one's stride is ldb
//    times the block sizes of the later ones, ldb the stride of the last;
//  * a K run (the contracted block, fixed sectors) of whole K-steps (16 f64 or
//    32 f32 rows);
//  * its last modes J modes whose contiguous run holds whole 16-byte chunks.
bool v_in_place_layout(const Plan& p, int64_t* ldb, bool* chunks) {
  if (p.cplx || p.v < 1 || p.t < 1 || p.subgroups) return false;
  // (with K stepped run by run, every step lies in one run and loads are single
  // elements: only the affine rows are needed)
  if (p.compute != SYMT_COMPUTE_F64 && p.compute != SYMT_COMPUTE_F32) return false;
  const int64_t elem = p.compute == SYMT_COMPUTE_F64 ? 8 : 4;
  const OperandDesc& V = p.V;
  int64_t st[kMaxOrder];
  int64_t a = 1;
  for (int m = V.n - 1; m >= 0; --m) { st[m] = a; a *= V.dims[m]; }
  const int64_t stride = st[p.posK_v[p.v - 1]];
  int64_t expect = stride;
  for (int i = p.v - 1; i >= 0; --i) {
    if (st[p.posK_v[i]] != expect) return false;
    expect *= V.dims[p.posK_v[i]];
  }
  int64_t run_j = 1;
  for (int i = p.t - 1; i >= 0 && st[p.posJ_v[i]] == run_j; --i) run_j *= V.dims[p.posJ_v[i]];
  const int64_t ve = 16 / elem, step = 128 / elem;
  const bool whole_chunks = run_j % ve == 0 && p.gn % ve == 0;
  if (chunks) *chunks = whole_chunks;
  if (p.krun == 0 && (p.nK % step != 0 || !whole_chunks)) return false;
  *ldb = stride;
  return true;
}

int make_plan(const char* einsum, const symt_group* group, const symt_tensor* u,
              const symt_tensor* v, const symt_tensor* w, int32_t compute, Plan* p,
              std::string* err) {
  if (!einsum || !p) return fail(err, SYMT_EINVAL, "einsum or plan is NULL");
  int rc = read_group(group, &p->g, err);
  if (rc) return rc;
  const bool force_steps = (compute & kForceSteps) != 0;
  compute &= ~kForceSteps;
  if (compute < SYMT_COMPUTE_F64 || compute > SYMT_COMPUTE_BF16X3)
    return fail(err, SYMT_EDTYPE, "unknown compute mode");
  p->compute = compute;

  // ---- parse "tu,tv->tw"
  std::string s(einsum);
  const size_t comma = s.find(',');
  const size_t arrow = s.find("->");
  if (comma == std::string::npos || arrow == std::string::npos || comma > arrow ||
      s.find(',', comma + 1) != std::string::npos || s.find("->", arrow + 2) != std::string::npos)
    return fail(err, SYMT_EEINSUM, "einsum must read \"u,v->w\"");
  p->tu = s.substr(0, comma);
  p->tv = s.substr(comma + 1, arrow - comma - 1);
  p->tw = s.substr(arrow + 2);
  for (const std::string* t : {&p->tu, &p->tv, &p->tw}) {
    if (t->empty() || t->size() > static_cast<size_t>(kMaxOrder))
      return fail(err, SYMT_EEINSUM, "einsum term empty or longer than 12 modes");
    for (size_t i = 0; i < t->size(); ++i) {
      if (!is_letter((*t)[i])) return fail(err, SYMT_EEINSUM, "einsum letters must be a-z/A-Z");
      if (t->find((*t)[i], i + 1) != std::string::npos)
        return fail(err, SYMT_EEINSUM, "letter repeated inside one einsum term");
    }
  }
  const std::string &tu = p->tu, &tv = p->tv, &tw = p->tw;
  std::string I, K, J;
  for (char c : tu) {
    const bool inv = tv.find(c) != std::string::npos, inw = tw.find(c) != std::string::npos;
    if (inv && inw) return fail(err, SYMT_EEINSUM, "a letter in all three terms is a batch index");
    if (!inv && !inw) return fail(err, SYMT_EEINSUM, "a letter of u appears nowhere else");
    (inw ? I : K).push_back(c);
  }
  for (char c : tv) {
    const bool inu = tu.find(c) != std::string::npos, inw = tw.find(c) != std::string::npos;
    if (!inu && !inw) return fail(err, SYMT_EEINSUM, "a letter of v appears nowhere else");
    if (!inu) J.push_back(c);
  }
  for (char c : tw)
    if (tu.find(c) == std::string::npos && tv.find(c) == std::string::npos)
      return fail(err, SYMT_EEINSUM, "a letter of the output appears in no input");
  if (tw.size() != I.size() + J.size())
    return fail(err, SYMT_EEINSUM, "output term must hold exactly the uncontracted letters");
  p->s = static_cast<int32_t>(I.size());
  p->v = static_cast<int32_t>(K.size());
  p->t = static_cast<int32_t>(J.size());

  // ---- operands
  if ((rc = read_operand(u, p->g, &p->U, "u", err))) return rc;
  if ((rc = read_operand(v, p->g, &p->V, "v", err))) return rc;
  p->cplx = is_complex(p->U.dtype);
  if (is_complex(p->V.dtype) != p->cplx)
    return fail(err, SYMT_EDTYPE, "u and v must both be complex or both be real");
  if ((rc = read_charges(u, p->g, &p->chg[0], "u", err))) return rc;
  if ((rc = read_charges(v, p->g, &p->chg[1], "v", err))) return rc;
  if (p->U.n != static_cast<int>(tu.size()) || p->V.n != static_cast<int>(tv.size()))
    return fail(err, SYMT_EINVAL, "operand order differs from its einsum term");
  for (int i = 0; i < p->s; ++i) p->posI_u[i] = static_cast<int32_t>(tu.find(I[i]));
  for (int i = 0; i < p->v; ++i) {
    p->posK_u[i] = static_cast<int32_t>(tu.find(K[i]));
    p->posK_v[i] = static_cast<int32_t>(tv.find(K[i]));
  }
  for (int i = 0; i < p->t; ++i) p->posJ_v[i] = static_cast<int32_t>(tv.find(J[i]));
  for (int i = 0; i < p->s; ++i) p->posI_w[i] = static_cast<int32_t>(tw.find(I[i]));
  for (int i = 0; i < p->t; ++i) p->posJ_w[i] = static_cast<int32_t>(tw.find(J[i]));

  // ---- contracted modes: equal block sizes and one sign ratio
  int sigma = 0;
  for (int i = 0; i < p->v; ++i) {
    if (p->U.dims[p->posK_u[i]] != p->V.dims[p->posK_v[i]])
      return fail(err, SYMT_EINVAL, "contracted mode '%s' has different block sizes",
                  std::string(1, K[i]).c_str());
    const int r = p->U.sign[p->posK_u[i]] * p->V.sign[p->posK_v[i]];
    if (sigma == 0) sigma = r;
    else if (r != sigma)
      return fail(err, SYMT_ESYM, "contracted modes carry mixed sign ratios c^V/c^U");
    for (int l = 0; l < p->g.size; ++l)
      if (table_at(p->chg[0], p->g.size, p->posK_u[i], l) != table_at(p->chg[1], p->g.size, p->posK_v[i], l))
        return fail(err, SYMT_ESYM, "contracted mode '%s' carries different charge tables in u and v",
                    std::string(1, K[i]).c_str());
    if (p->U.hs[p->posK_u[i]] != p->V.hs[p->posK_v[i]])
      return fail(err, SYMT_ESYM, "contracted mode '%s' has different sector counts in u and v",
                  std::string(1, K[i]).c_str());
  }
  // subgroup modes (fewer than |G| sectors): cyclic groups, no charge tables
  for (int m = 0; m < p->U.n; ++m) p->subgroups = p->subgroups || p->U.hs[m] != p->g.size;
  for (int m = 0; m < p->V.n; ++m) p->subgroups = p->subgroups || p->V.hs[m] != p->g.size;
  if (p->subgroups && (p->g.nf != 1 || !p->chg[0].empty() || !p->chg[1].empty()))
    return fail(err, SYMT_EUNSUPPORTED, "subgroup modes need a cyclic group and no charge tables");
  // v = 0 (outer product): no ratio is defined; -1 makes W's coefficients u's
  // followed by v's and Z^W = Z^U + Z^V
  p->sigma = p->v == 0 ? -1 : sigma;
  if (p->v == 0 && w && w->signs && w->nmodes == static_cast<int32_t>(tw.size()) &&
      strnlen(w->signs, tw.size()) == tw.size()) {
    // An outer product's nonzero blocks satisfy u's and v's rules each on its
    // own, so the rule derived with sigma = +1 describes them as well (it is
    // u's rule when v is an operand's gradient partner, as in dU = dW (x) V):
    // take +1 when the given output carries that rule and not the -1 one.
    auto matches = [&](int sg) {
      const int zc = gsub(p->g, p->U.charge, gtimes(p->g, sg, p->V.charge));
      bool same = w->charge == zc, flipped = w->charge == gneg(p->g, zc);
      for (size_t m = 0; m < tw.size(); ++m) {
        const size_t pu = tu.find(tw[m]);
        const int c = (pu != std::string::npos) ? p->U.sign[pu] : -sg * p->V.sign[tv.find(tw[m])];
        const int given = w->signs[m] == '+' ? 1 : w->signs[m] == '-' ? -1 : 0;
        same = same && given == c;
        flipped = flipped && given == -c;
      }
      return same || flipped;
    };
    if (!matches(-1) && matches(+1)) p->sigma = 1;
  }
  sigma = p->sigma;

  // ---- derived output rule: c^W = (c^U_I, -sigma c^V_J), Z^W = Z^U - sigma Z^V
  for (size_t m = 0; m < tw.size(); ++m) {
    const char c = tw[m];
    const size_t pu = tu.find(c);
    p->w_sign[m] = (pu != std::string::npos) ? p->U.sign[pu] : -sigma * p->V.sign[tv.find(c)];
  }
  p->w_charge = gsub(p->g, p->U.charge, gtimes(p->g, sigma, p->V.charge));
  // With an empty mode group one generalized delta fixes Q: delta(2) with no K
  // modes gives Q = 0, delta(1) with no I modes Q = Z^U, delta(3) with no J
  // modes sigma Q = Z^V.  Only that slice of the aligned forms is nonzero.
  p->q_pin = p->v == 0 ? 0 : p->s == 0 ? p->U.charge : p->t == 0 ? gtimes(p->g, sigma, p->V.charge) : -1;
  {
    // The sum of a delta's terms ranges over the subgroup generated by its
    // coefficients' magnitudes (multiples of their gcd d with |G|), or is 0 for
    // an empty sum (d = |G|).  A Q for which one of the three deltas cannot
    // hold has an all-zero slice in the aligned forms and is skipped.
    const int G = p->g.size;
    auto gcd_of = [&](const OperandDesc& X, const int32_t* pos, int count) {
      if (count == 0) return G;
      int d = G;
      for (int i = 0; i < count; ++i) d = std::gcd(d, G / X.hs[pos[i]]);
      return d;
    };
    const int dI = gcd_of(p->U, p->posI_u, p->s), dK = gcd_of(p->U, p->posK_u, p->v),
              dJ = gcd_of(p->V, p->posJ_v, p->t);
    auto reach = [&](int x, int d) { return d == 1 || (d == G ? x == 0 : x % d == 0); };
    std::vector<int> live;
    for (int q = 0; q < G; ++q)
      if (reach(gsub(p->g, p->U.charge, q), dI) && reach(q, dK) &&
          reach(gsub(p->g, p->V.charge, gtimes(p->g, sigma, q)), dJ))
        live.push_back(q);
    p->nq = static_cast<int64_t>(live.size());
    p->q0 = live.empty() ? 0 : live[0];
    p->q_step = live.size() > 1 ? live[1] - live[0] : 1;
    for (size_t i = 0; i < live.size(); ++i)
      if (live[i] != p->q0 + static_cast<int>(i) * p->q_step) {   // not a progression: move every slice
        p->q0 = 0, p->q_step = 1, p->nq = G;
        break;
      }
  }
  // derived charge tables: u's rows on I modes, v's on J modes
  std::vector<int32_t> w_chg;
  if (!p->chg[0].empty() || !p->chg[1].empty()) {
    const int G = p->g.size;
    w_chg.resize(tw.size() * static_cast<size_t>(G));
    bool identity = true;
    for (size_t m = 0; m < tw.size(); ++m) {
      const char c = tw[m];
      const size_t pu = tu.find(c);
      for (int l = 0; l < G; ++l) {
        const int32_t x = pu != std::string::npos ? table_at(p->chg[0], G, static_cast<int>(pu), l)
                                                   : table_at(p->chg[1], G, static_cast<int>(tv.find(c)), l);
        w_chg[m * G + l] = x;
        identity = identity && x == l;
      }
    }
    if (identity) w_chg.clear();
  }

  // ---- output descriptor
  p->has_w = (w != nullptr);
  if (w) {
    if ((rc = read_operand(w, p->g, &p->W, "w", err))) return rc;
    if (is_complex(p->W.dtype) != p->cplx)
      return fail(err, SYMT_EDTYPE, "w must be complex exactly when u and v are");
    if (p->W.n != static_cast<int>(tw.size()))
      return fail(err, SYMT_EINVAL, "output order differs from its einsum term");
    for (size_t m = 0; m < tw.size(); ++m) {
      const char c = tw[m];
      const size_t pu = tu.find(c);
      const int64_t d = (pu != std::string::npos) ? p->U.dims[pu] : p->V.dims[tv.find(c)];
      if (p->W.dims[m] != d) return fail(err, SYMT_EINVAL, "output block sizes differ from inputs'");
      const int32_t h = (pu != std::string::npos) ? p->U.hs[pu] : p->V.hs[tv.find(c)];
      if (p->W.hs[m] != h)
        return fail(err, SYMT_ESYM, "output sector counts differ from u's (I modes) and v's (J modes)");
    }
    bool same = p->W.charge == p->w_charge, flipped = p->W.charge == gneg(p->g, p->w_charge);
    for (size_t m = 0; m < tw.size(); ++m) {
      same = same && p->W.sign[m] == p->w_sign[m];
      flipped = flipped && p->W.sign[m] == -p->w_sign[m];
    }
    if (!same && !flipped)
      return fail(err, SYMT_ESYM, "output signs/charge differ from the rule implied by u and v");
    std::vector<int32_t> given;
    if ((rc = read_charges(w, p->g, &given, "w", err))) return rc;
    if (given != w_chg)
      return fail(err, SYMT_ESYM, "output charge tables differ from u's (I modes) and v's (J modes)");
  } else {
    p->W = OperandDesc{};
    p->W.n = static_cast<int32_t>(tw.size());
    for (size_t m = 0; m < tw.size(); ++m) {
      const size_t pu = tu.find(tw[m]);
      p->W.hs[m] = (pu != std::string::npos) ? p->U.hs[pu] : p->V.hs[tv.find(tw[m])];
    }
    int64_t e = 1;
    for (int m = 0; m < p->W.n - 1; ++m) mul_ok(e, p->W.hs[m], &e);
    for (size_t m = 0; m < tw.size(); ++m) {
      const char c = tw[m];
      const size_t pu = tu.find(c);
      p->W.dims[m] = (pu != std::string::npos) ? p->U.dims[pu] : p->V.dims[tv.find(c)];
      p->W.sign[m] = p->w_sign[m];
      if (!mul_ok(e, p->W.dims[m], &e)) return fail(err, SYMT_EINVAL, "output size overflows");
    }
    p->W.charge = p->w_charge;
    p->W.dtype = p->cplx ? SYMT_C128 : SYMT_F64;
    p->W.elems = e;
  }
  p->chg[2] = w_chg;
  p->charges = !p->chg[0].empty() || !p->chg[1].empty() || !p->chg[2].empty();

  // ---- aligned shapes M = G^(s-1) n_I, Kd = G^(v-1) n_K, N = G^(t-1) n_J (each
  // G factor is a stored mode's sector count: the group's modes but its last)
  p->nI = p->nK = p->nJ = 1;
  for (int i = 0; i < p->s; ++i) mul_ok(p->nI, p->U.dims[p->posI_u[i]], &p->nI);
  for (int i = 0; i < p->v; ++i) mul_ok(p->nK, p->U.dims[p->posK_u[i]], &p->nK);
  for (int i = 0; i < p->t; ++i) mul_ok(p->nJ, p->V.dims[p->posJ_v[i]], &p->nJ);
  int64_t gs = 1, gt = 1, gv = 1;
  for (int i = 0; i + 1 < p->s; ++i) mul_ok(gs, p->U.hs[p->posI_u[i]], &gs);
  for (int i = 0; i + 1 < p->t; ++i) mul_ok(gt, p->V.hs[p->posJ_v[i]], &gt);
  for (int i = 0; i + 1 < p->v; ++i) mul_ok(gv, p->U.hs[p->posK_u[i]], &gv);
  if (!mul_ok(gs, p->nI, &p->M) || !mul_ok(gv, p->nK, &p->Kd) || !mul_ok(gt, p->nJ, &p->N))
    return fail(err, SYMT_EINVAL, "aligned shape overflows");
  // complex: the real representation doubles the contracted and output columns
  p->gk = p->cplx ? 2 * p->Kd : p->Kd;
  p->gn = p->cplx ? 2 * p->N : p->N;
  // the split-bf16 products read K in 16-byte chunks of 8: the contraction's
  // workspace planes take a zero pad up to a multiple of 8 (the standalone
  // aligned layouts keep K unpadded)
  p->kpad = compute == SYMT_COMPUTE_BF16X3 ? (p->gk + 7) / 8 * 8 : p->gk;
  // ... and up to a multiple of 32 where a wide tile multiplies them (32-deep
  // K-steps), if that adds at most an eighth of K
  if (compute == SYMT_COMPUTE_BF16X3 && p->kpad % 32 != 0 && p->nq > 0 && p->M > 0 && p->gn > 0) {
    const char* tile_env = std::getenv("SYMT_GEMM_TILE");
    const std::string tile = tile_env ? tile_env : "";
    const int64_t k32 = (p->gk + 31) / 32 * 32;
    const bool wide = tile.empty() ? bf16x3_wide_tile(p->nq, p->M, p->gn) >= 0
                                   : tile == "bw256x256s2" || tile == "bw256x128s3";
    if (wide && 8 * (k32 - p->gk) <= p->gk) p->kpad = k32;
  }
  if (p->M > INT32_MAX || p->gn > INT32_MAX || p->gk > INT32_MAX)
    return fail(err, SYMT_EUNSUPPORTED, "aligned matrix dimension above 2^31-1");
  p->flops = 2.0 * static_cast<double>(p->nq) * static_cast<double>(p->M) * static_cast<double>(p->gk) *
             static_cast<double>(p->gn);

  // ---- buffer sizes for the compute mode.  The aligned forms hold |G| M K,
  // |G| K N and |G| M N reals (K and N of the real product); with Q pinned the
  // contraction keeps only the one nonzero slice of each in its workspace.
  int64_t au = 0, av = 0, aw = 0;
  if (!mul_ok(p->M, p->gk, &au) || !mul_ok(au, p->g.size, &au) || !mul_ok(p->gk, p->gn, &av) ||
      !mul_ok(av, p->g.size, &av) || !mul_ok(p->M, p->gn, &aw) || !mul_ok(aw, p->g.size, &aw))
    return fail(err, SYMT_EINVAL, "aligned form size overflows");
  const size_t ea = compute == SYMT_COMPUTE_F64 ? 8 : 4, ec = compute == SYMT_COMPUTE_F32 ? 4 : 8;
  p->bytes_u_al = ea * static_cast<size_t>(au);
  p->bytes_v_al = ea * static_cast<size_t>(av);
  p->bytes_w_al = ec * static_cast<size_t>(aw);
  const size_t G = static_cast<size_t>(p->g.size), nq = static_cast<size_t>(p->nq);
  p->ws_u_al = ea * static_cast<size_t>(p->M) * static_cast<size_t>(p->kpad) * nq;
  p->ws_v_al = ea * static_cast<size_t>(p->kpad) * static_cast<size_t>(p->gn) * nq;
  p->ws_w_al = p->bytes_w_al / G * nq;
  p->workspace = round_up(p->ws_u_al, 256) + round_up(p->ws_v_al, 256) + round_up(p->ws_w_al, 256);

  // ---- fused product: A read from U's standard form along contiguous K runs
  // (U's last v modes are its contracted modes and their block holds whole
  // K-depths), C written straight into W's standard form.
  // Complex operands read and write their interleaved pairs as reals (a K run
  // of nK pairs is 2 nK reals).  Every product tile reads one K-step from one
  // run: 16 reals on the register tiles, one 128-byte row (16 f64 or 32 f32)
  // on the global-to-LDS tiles.
  const int want = p->cplx ? (compute == SYMT_COMPUTE_F64 ? SYMT_C128 : SYMT_C64)
                           : (compute == SYMT_COMPUTE_F64 ? SYMT_F64 : SYMT_F32);
  bool trailing_k = true;
  for (int i = 0; i < p->v; ++i) trailing_k = trailing_k && p->posK_u[i] == p->U.n - p->v + i;
  {
    // U's contracted modes from its fastest one down, while they nest (a contiguous K run)
    int64_t st[kMaxOrder];
    int64_t a = 1;
    for (int m = p->U.n - 1; m >= 0; --m) { st[m] = a; a *= p->U.dims[m]; }
    p->u_k_run = 1;
    for (int i = p->v - 1; i >= 0 && st[p->posK_u[i]] == p->u_k_run; --i) p->u_k_run *= p->U.dims[p->posK_u[i]];
  }
  // A single run (one contracted mode, or every contracted sector fixed) holds
  // any K-step; the product masks the steps past its end.
  const int64_t run = (p->cplx ? 2 : 1) * p->nK;
  const int64_t step = 128 / (compute == SYMT_COMPUTE_F64 ? 8 : 4);
  const bool whole_aligned = run % kFpBK == 0 && run % step == 0;
  const bool whole_steps = whole_aligned || run == p->gk;
  const bool fp_ok = compute != SYMT_COMPUTE_BF16X3 && p->U.dtype == want && (!w || p->W.dtype == want) &&
                     whole_steps;
  // split-bf16: the register-staged tiles read U (binary64 or binary32) along
  // 32-deep K-steps and split it into hi/lo in registers; W takes the binary64
  // sums (rounded to binary32 for a binary32 W)
  const bool bf_ok = compute == SYMT_COMPUTE_BF16X3 && !p->cplx &&
                     (p->U.dtype == SYMT_F64 || p->U.dtype == SYMT_F32) &&
                     (!w || p->W.dtype == SYMT_F64 || p->W.dtype == SYMT_F32) &&
                     run % 32 == 0 && bf16x3_register_tile(p->M, p->gn, p->gk);
  // K runs that do not hold whole K-steps: where the product runs on register
  // tiles anyway, they step each run on their own (masking its last step), so A
  // is still read in place (and V, with one-element loads); global-to-LDS shapes
  // keep the aligned forms.  A single such run is stepped the same way.
  const bool stepped = !whole_aligned && compute != SYMT_COMPUTE_BF16X3 && !p->cplx && p->U.dtype == want &&
                       (!w || p->W.dtype == want) && p->nK <= INT32_MAX && p->nK > 0 &&
                       p->gk % p->nK == 0 &&
                       !choose_fp_gemm(p->g.size, p->M, p->gn, p->gk, static_cast<int>(ea), true).dma;
  // U's contracted modes are not its last ones: A is loaded K-major straight from U
  // (row k of a K-step at its own column-table entry, M chunks along U's other
  // modes), as B is from V: on register tiles, and on the 128-row global-to-LDS
  // tiles where U's last modes hold whole 16-byte chunks along M.
  bool a_chunks = false;
  {
    // contiguous run of U's output modes at its end (16-byte loads along M)
    int64_t st[kMaxOrder];
    int64_t a = 1;
    for (int m = p->U.n - 1; m >= 0; --m) { st[m] = a; a *= p->U.dims[m]; }
    int64_t i_run = 1;
    for (int i = p->s - 1; i >= 0 && st[p->posI_u[i]] == i_run; --i) i_run *= p->U.dims[p->posI_u[i]];
    // (complex: pairs interleave, one-element loads)
    a_chunks = !p->cplx && i_run % (16 / static_cast<int64_t>(ea)) == 0;
  }
  // (where the model's global-to-LDS tile is a 96-row one, which cannot read
  // K-major A, a 128-row one replaces it only for a U large enough that aligning
  // it would cost more than the other tile: 64 MiB; else U is aligned first)
  const GemmChoice g_any = choose_fp_gemm(p->g.size, p->M, p->gn, p->gk, static_cast<int>(ea), true);
  const GemmChoice g_at = choose_fp_gemm(p->g.size, p->M, p->gn, p->gk, static_cast<int>(ea), true, true);
  const bool at_dma = g_at.dma && a_chunks &&
                      (g_at.tile == g_any.tile || static_cast<double>(ea) * p->U.elems >= 64.0 * (1 << 20));
  const bool at_ok = !trailing_k && compute != SYMT_COMPUTE_BF16X3 && p->U.dtype == want &&
                     (!w || p->W.dtype == want) && (!g_any.dma || at_dma);
  p->fused = !force_steps && !p->subgroups && p->nq == p->g.size &&
             (((fp_ok || bf_ok || stepped) && trailing_k) || at_ok) &&
             p->M > 0 && p->N > 0 && p->Kd > 0 && p->U.elems > 0;
  p->a_trans = p->fused && !trailing_k;
  p->krun = p->fused && stepped ? static_cast<int32_t>(p->nK) : 0;
  if (p->a_trans) p->a_chunks = a_chunks;
  // Otherwise, for W in the compute type (complex: its complex counterpart), U
  // alone is aligned and the same product reads U_al through affine tables (in
  // reals), V in place where it can, and writes W in place.
  // (split-bf16: U and V go to hi/lo planes as in three steps, and the product
  // writes its binary64 sums straight into W)
  const int w_want = compute == SYMT_COMPUTE_F32 ? SYMT_F32 : SYMT_F64;
  // W's aligned columns: the contiguous run of its output modes from V (the
  // split-bf16 epilogue only pays off where its column stores coalesce; with
  // W's columns transposed, the W transform's LDS-tiled transpose is cheaper)
  int64_t w_run = 1;
  {
    int64_t st[kMaxOrder];
    int64_t a = 1;
    for (int m = p->W.n - 1; m >= 0; --m) { st[m] = a; a *= p->W.dims[m]; }
    for (int i = p->t - 1; i >= 0 && st[p->posJ_w[i]] == w_run; --i) w_run *= p->W.dims[p->posJ_w[i]];
    int64_t r_run = 1;
    for (int i = p->s - 1; i >= 0 && st[p->posI_w[i]] == r_run; --i) r_run *= p->W.dims[p->posI_w[i]];
    p->w_col_run = w_run;
    p->w_row_run = r_run;
  }
  p->fused_ua = !p->fused && !force_steps && !p->subgroups && p->nq == p->g.size &&
                (!w || p->W.dtype == (p->cplx ? want : w_want) ||
                 (compute == SYMT_COMPUTE_BF16X3 && p->W.dtype == SYMT_F32)) &&
                p->M > 0 && p->N > 0 && p->Kd > 0 && p->U.elems > 0 &&
                (compute != SYMT_COMPUTE_BF16X3 || (w_run >= 16 && !p->cplx));
  if (p->fused || p->fused_ua) {
    const size_t G = static_cast<size_t>(p->g.size);
    p->bytes_tables = round_up(8 * G * p->M, 256) * 2 + round_up(8 * G * p->gk, 256) +
                      round_up(8 * G * p->gn, 256);
    p->workspace = (p->fused_ua ? round_up(p->ws_u_al, 256) : 0) + round_up(p->ws_v_al, 256) + p->bytes_tables;
  }
  // ---- V read in place as well (see v_in_place_layout); V_al keeps its place in
  // the workspace: a V that is not 16-byte aligned is aligned as before.
  int64_t ldb = 0;
  const char* vip_env = std::getenv("SYMT_FUSED_V");
  const bool vip_off = vip_env && std::atoi(vip_env) == 0;
  bool chunks = false;
  if (!vip_off && (p->fused || p->fused_ua) && !p->cplx && p->V.dtype == want &&
      v_in_place_layout(*p, &ldb, &chunks)) {
    const size_t G = static_cast<size_t>(p->g.size);
    p->fused_b = true;
    p->fused_b_chunks = chunks;
    p->ldb = ldb;
    p->bytes_tables += round_up(8 * G * p->gk, 256) + round_up(8 * G * p->gn, 256);
    p->workspace = (p->fused_ua ? round_up(p->ws_u_al, 256) : 0) + round_up(p->ws_v_al, 256) + p->bytes_tables;
  }
  // ---- split-bf16 planes interleaved by K-steps where the wide tiles multiply
  // both aligned operands (the launcher's own pick, or a forced wide tile);
  // SYMT_BF16_IL=0 keeps the plane-after-plane layout (tuning and tests)
  if (compute == SYMT_COMPUTE_BF16X3 && !p->cplx && !p->fused && !p->fused_b && p->nq > 0 && p->M > 0 &&
      p->gn > 0 && p->kpad % 32 == 0) {
    const char* tile_env = std::getenv("SYMT_GEMM_TILE");
    const std::string tile = tile_env ? tile_env : "";
    const char* il_env = std::getenv("SYMT_BF16_IL");
    const bool wide = tile.empty() ? bf16x3_wide_tile(p->nq, p->M, p->gn) >= 0
                                   : tile == "bw256x256s2" || tile == "bw256x128s3";
    p->bf16_il = wide && !(il_env && std::atoi(il_env) == 0);
    const char* fa_env = std::getenv("SYMT_BF16_FA");
    const bool wide256 = tile.empty() ? bf16x3_wide_tile(p->nq, p->M, p->gn) == 0 : tile == "bw256x256s2";
    p->bf16_wide_fa = p->bf16_il && wide256 && p->fused_ua && p->U.dtype == SYMT_F32 && trailing_k &&
                      p->nK % 4 == 0 && p->gk == p->kpad && !(fa_env && std::atoi(fa_env) == 0);
  }
  if (p->charges) {
    p->bytes_charges = 4 * 2 * static_cast<size_t>(p->g.size) * (p->U.n + p->V.n + p->W.n);
  }
  // Room for stream-K pieces when the model would pick it on 16-byte aligned operands.
  if (compute != SYMT_COMPUTE_BF16X3 && p->nq > 0 && p->M > 0 && p->gn > 0 && p->gk > 0) {
    const GemmChoice gc = choose_fp_gemm(p->nq, p->M, p->gn, p->gk,
                                         compute == SYMT_COMPUTE_F64 ? 8 : 4, true, p->a_trans);
    p->bytes_partial = gc.partial_bytes;
    p->workspace += round_up(p->bytes_partial, 256);
  }
  p->workspace += round_up(p->bytes_charges, 256);
  return SYMT_OK;
}

std::vector<int32_t> charge_tables_device(const Plan& p, int64_t offset[3]) {
  const int G = p.g.size;
  const int n[3] = {p.U.n, p.V.n, p.W.n};
  std::vector<int32_t> out;
  for (int op = 0; op < 3; ++op) {
    offset[op] = static_cast<int64_t>(out.size());
    for (int m = 0; m < n[op]; ++m) {
      const size_t base = out.size();
      out.resize(base + 2 * static_cast<size_t>(G));
      for (int l = 0; l < G; ++l) {
        const int32_t c = table_at(p.chg[op], G, m, l);
        out[base + l] = c;
        out[base + G + c] = l;
      }
    }
  }
  return out;
}

namespace {
struct FpTile {
  const char* name;
  int bm, bn;
  bool dma;
  double eff64, eff32;   // measured MFMA efficiency on a large, evenly tiled product
  int wgs;               // resident workgroups per CU (global-to-LDS tiles)
};
// Efficiencies: 16 x 6144 x 2048 x 1152, a whole number of 256-tile waves for
// every tile; f64 and f32.
constexpr FpTile kFpTiles[] = {
    {"128x128", 128, 128, false, 0.78, 0.78, 0},  {"128x96", 128, 96, false, 0.75, 0.79, 0},
    {"128x64", 128, 64, false, 0.72, 0.78, 0},    {"128x48", 128, 48, false, 0.74, 0.75, 0},
    {"96x96", 96, 96, false, 0.72, 0.77, 0},      {"64x96", 64, 96, false, 0.73, 0.76, 0},
    {"d128x128s2", 128, 128, true, 0.87, 0.85, 2}, {"d128x96s2", 128, 96, true, 0.86, 0.84, 2},
    {"d128x64s3", 128, 64, true, 0.84, 0.78, 2},  {"d96x96s3", 96, 96, true, 0.86, 0.84, 2},
    // two stages: 48 KB of LDS, three workgroups (three waves per SIMD) per CU
    {"d96x96s2", 96, 96, true, 0.875, 0.84, 3},
};
// Stream-K keeps this share of a tile's steady-state efficiency (B panels are
// fetched at staggered K positions, pieces and their fixup); measured on the
// CCD ladder over Z_8.
constexpr double kSkEff64 = 0.965, kSkEff32 = 0.80;
// Resident workgroups per CU that a register tile needs to reach its measured
// efficiency (the efficiencies above come from launches of many tiles per CU).
constexpr int64_t kRegSaturation = 3;
constexpr int kNumFpTiles = sizeof(kFpTiles) / sizeof(kFpTiles[0]);
}  // namespace

// Time model: a tile costs 2*bm*bn*K flops at its measured efficiency of one
// CU's share of the MFMA peak.  Data-parallel launches pay whole waves of 256
// tiles; stream-K pays the exact fraction plus writing and re-reading the
// pieces of cut tiles (at most two per persistent workgroup), their pipeline
// fills (~1.5 us each), and one more launch (~5 us).
namespace {
GemmChoice choose_among(int64_t batch, int64_t M, int64_t N, int64_t K, int elem, bool aligned,
                        const char* forced, int sk_mode, bool a_kmajor) {
  auto usable = [&](const FpTile& t) {
    if (!t.dma) return true;
    return aligned && K % (128 / elem) == 0 && N % (16 / elem) == 0 && (t.bn * elem / 16) % 16 == 0 &&
           (!a_kmajor || (t.bm == 128 && M % (16 / elem) == 0));
  };
  const double per_cu = (elem == 8 ? 78.6e12 : 157.3e12) / 256.0;
  const bool big = 2.0 * static_cast<double>(batch) * M * N * K >= 1e9;
  GemmChoice best;
  // K and N at most 64: 2 K N flops per 8 (K + N) bytes of A and C, bound by HBM
  // on any tile; the row-streaming product reads A once and keeps B in LDS
  // (named "rows"; it needs enough rows to spread over the device)
  // M and N at most 64 with a long K: 2 M N flops per 8 (M + N) bytes, HBM
  // bound, and most of any 128-wide tile would be padding; the long-K product
  // splits K over ranges and sums their partials in order (named "tallk")
  const bool tallk_forced = forced && std::strcmp(forced, "tallk") == 0;
  if (M >= 1 && M <= 64 && N >= 1 && N <= 64 && K >= 1 && batch >= 1 && batch <= 65535 && K <= INT32_MAX &&
      (tallk_forced || (!forced && K >= 1024 && sk_mode != 0))) {
    best.tile = kTallKTile;
    best.bm = static_cast<int>(M);
    best.bn = static_cast<int>(N);
    best.splits = tallk_ranges(batch, K);
    best.partial_bytes = static_cast<size_t>(batch) * best.splits * M * N * elem;
    return best;
  }
  const bool rows_forced = forced && std::strcmp(forced, "rows") == 0;
  if (K >= 1 && K <= 64 && N >= 1 && N <= 64 && batch >= 1 && batch <= 65535 && M >= 1 &&
      (rows_forced || (!forced && batch * M >= 16384))) {
    best.tile = kRowsTile;
    best.bm = 32;
    best.bn = static_cast<int>(N);
    return best;
  }
  double best_t = 0;
  for (int i = 0; i < kNumFpTiles; ++i) {
    const FpTile& t = kFpTiles[i];
    if (!usable(t)) continue;
    if (forced && std::strcmp(forced, t.name) != 0) continue;
    const int64_t tiles = batch * ((M + t.bm - 1) / t.bm) * ((N + t.bn - 1) / t.bn);
    const double eff = elem == 8 ? t.eff64 : t.eff32;
    const double t_tile = 2.0 * t.bm * t.bn * static_cast<double>(K) / (eff * per_cu);
    for (int sk = 0; sk < 2; ++sk) {
      if (sk && (!t.dma || sk_mode == 0)) continue;
      if (!sk && t.dma && sk_mode == 1) continue;
      double time;
      size_t partial = 0;
      if (!sk) {
        // register tiles hide their load latency with about three resident
        // workgroups per CU: fewer tiles than that still take three tiles' time
        // (on products of a GFLOP and up; below, launches dominate)
        const int64_t rounds = (tiles + 255) / 256;
        time = static_cast<double>(t.dma || !big ? rounds : std::max<int64_t>(rounds, kRegSaturation)) * t_tile;
      } else {
        partial = 2 * static_cast<size_t>(std::min(kSkSlots, 256 * t.wgs)) * t.bm * t.bn * elem;
        time = static_cast<double>(tiles) / 256.0 * t_tile / (elem == 8 ? kSkEff64 : kSkEff32) +
               2.0 * static_cast<double>(partial) / 5e12 +
               2 * 1.5e-6 + 5e-6;
      }
      if (best.tile < 0 || time < best_t) {
        best.tile = i; best.bm = t.bm; best.bn = t.bn; best.dma = t.dma; best.sk = sk;
        best.splits = 1;
        best.partial_bytes = partial;
        best_t = time;
      }
    }
    // Register tiles with few tiles and a long K: split each tile's K-steps into
    // runs for more workgroups (about two per CU), summed in order afterwards.
    // Each run pays a pipeline fill of about two K-steps.
    if (!t.dma && sk_mode != 0) {
      const int64_t nk = (K + 15) / 16;
      const int64_t sp = std::min<int64_t>({(256 * kRegSaturation + tiles - 1) / std::max<int64_t>(tiles, 1),
                                            nk / 8, 128});
      if (sp > 1) {
        const size_t partial = static_cast<size_t>(tiles * sp) * t.bm * t.bn * elem;
        const int64_t rounds = std::max<int64_t>((tiles * sp + 255) / 256, big ? kRegSaturation : 1);
        const double time = static_cast<double>(rounds) * t_tile / static_cast<double>(sp) *
                                (1.0 + 2.0 * static_cast<double>(sp) / static_cast<double>(nk)) +
                            2.0 * static_cast<double>(partial) / 5e12 + 5e-6;
        if (time < best_t) {
          best.tile = i; best.bm = t.bm; best.bn = t.bn; best.dma = false; best.sk = false;
          best.splits = static_cast<int>(sp);
          best.partial_bytes = partial;
          best_t = time;
        }
      }
    }
  }
  return best;
}
}  // namespace

bool tallk_groups(const Plan& p) {
  if (p.cplx || (p.compute != SYMT_COMPUTE_F64 && p.compute != SYMT_COMPUTE_F32)) return false;
  const int64_t elem = p.compute == SYMT_COMPUTE_F64 ? 8 : 4;
  const int64_t group = 16, ve = 16 / elem;
  // (U's K order ends with its trailing contracted modes: u_k_run of them are contiguous)
  const bool a_ok = p.fused_ua ? p.kpad % group == 0 : p.fused && p.u_k_run % group == 0;
  const bool b_ok = p.fused_b ? p.nK % group == 0 && p.fused_b_chunks : p.gn % ve == 0;
  return a_ok && b_ok;
}

// SYMT_GEMM_TILE=<name> restricts the choice to one tile (ignored where it does
// not apply); SYMT_GEMM_SK=0 forbids stream-K and split K, 1 forces stream-K on
// the DMA tiles.
GemmChoice choose_fp_gemm(int64_t batch, int64_t M, int64_t N, int64_t K, int elem, bool aligned,
                          bool a_kmajor) {
  const char* forced = std::getenv("SYMT_GEMM_TILE");
  const char* sk_env = std::getenv("SYMT_GEMM_SK");
  const int sk_mode = sk_env ? std::atoi(sk_env) : -1;
  GemmChoice g = choose_among(batch, M, N, K, elem, aligned, forced, sk_mode, a_kmajor);
  if (g.tile < 0) g = choose_among(batch, M, N, K, elem, aligned, nullptr, sk_mode, a_kmajor);
  return g;
}

// The split-bf16 launcher's choice: SYMT_GEMM_TILE may name one of its tiles;
// by default global-to-LDS tiles where K holds whole 32-deep steps and the
// product is at least 256 x 512.
bool bf16x3_register_tile(int64_t M, int64_t N, int64_t K) {
  const char* forced = std::getenv("SYMT_GEMM_TILE");
  const std::string f = forced ? forced : "";
  const bool dma_ok = K % 32 == 0;
  if ((f == "bd256x128s3" || f == "bd128x256s3" || f == "bw256x256s2" || f == "bw256x128s3") && dma_ok)
    return false;
  if (f == "b128x128k64" || f == "b128x128k32" || f == "b256x128k32" || f == "b128x256k32" ||
      f == "b128x64k32" || f == "b128x96k32" || f == "b64x64k32")
    return true;
  return !(dma_ok && M >= 256 && N >= 512);
}

int bf16x3_wide_tile(int64_t batch, int64_t M, int64_t N) {
  if (M < 256) return -1;
  for (int v = 0; v < 2; ++v) {
    const int64_t bn = v == 0 ? 256 : 128;
    if (N < bn) continue;
    const int64_t tn = (N + bn - 1) / bn;
    if (8 * (tn * bn - N) > N) continue;                       // padded columns above 1/8
    if (batch * ((M + 255) / 256) * tn < 256) continue;        // fewer tiles than CUs
    return v;
  }
  return -1;
}

int bf16x3_fused_tile(int64_t M, int64_t N) {
  const char* forced = std::getenv("SYMT_GEMM_TILE");
  const std::string f = forced ? forced : "";
  if (f == "b128x64k32") return 0;
  if (f == "b128x256k32") return 2;
  if (f == "b128x128k32") return 1;
  if (f == "b128x96k32") return 3;
  if (N <= 64) return 0;
  if (N >= 1024 && M >= 1024) return 2;
  return 1;
}

namespace {
// Sector groups of an operand (rows, cols) with their deltas; shared by the
// transform and offset-table descriptors.
void sector_groups(const Plan& p, int operand, SectorGroup* R, SectorGroup* C) {
  if (operand == 0) {
    R->count = p.s;
    for (int i = 0; i < p.s; ++i) { R->pos[i] = p.posI_u[i]; R->coef[i] = p.U.sign[p.posI_u[i]]; }
    R->alpha = -1; R->beta = p.U.charge;                 // delta(1): sum c^U_I I + Q == Z^U
    C->count = p.v;
    for (int i = 0; i < p.v; ++i) { C->pos[i] = p.posK_u[i]; C->coef[i] = p.U.sign[p.posK_u[i]]; }
    C->alpha = 1; C->beta = 0;                           // delta(2): sum c^U_K K == Q
  } else if (operand == 1) {
    R->count = p.v;
    for (int i = 0; i < p.v; ++i) { R->pos[i] = p.posK_v[i]; R->coef[i] = p.U.sign[p.posK_u[i]]; }
    R->alpha = 1; R->beta = 0;                           // delta(2), U's coefficients
    C->count = p.t;
    for (int i = 0; i < p.t; ++i) { C->pos[i] = p.posJ_v[i]; C->coef[i] = p.V.sign[p.posJ_v[i]]; }
    C->alpha = -p.sigma; C->beta = p.V.charge;           // delta(3): sum c^V_J J + sigma Q == Z^V
  } else {
    R->count = p.s;
    for (int i = 0; i < p.s; ++i) { R->pos[i] = p.posI_w[i]; R->coef[i] = p.U.sign[p.posI_u[i]]; }
    R->alpha = -1; R->beta = p.U.charge;
    C->count = p.t;
    for (int i = 0; i < p.t; ++i) { C->pos[i] = p.posJ_w[i]; C->coef[i] = p.V.sign[p.posJ_v[i]]; }
    C->alpha = -p.sigma; C->beta = p.V.charge;
  }
  // sector counts of the members (subgroup modes: H < |G|, coefficient magnitude |G|/H)
  const OperandDesc& X = operand == 0 ? p.U : operand == 1 ? p.V : p.W;
  for (SectorGroup* sg : {R, C})
    for (int i = 0; i < sg->count; ++i) {
      sg->rad[i] = X.hs[sg->pos[i]];
      sg->mag[i] = p.g.size / sg->rad[i];
    }
}
}  // namespace

OffsetParams make_offsets(const Plan& p, int operand, bool rows) {
  OffsetParams o;
  std::memset(&o, 0, sizeof o);     // chg (charge tables) stays nullptr until launch
  o.g = p.g;
  SectorGroup R, C;
  sector_groups(p, operand, &R, &C);
  o.grp = rows ? R : C;
  const OperandDesc& X = operand == 0 ? p.U : operand == 1 ? p.V : p.W;
  int64_t std_stride[kMaxOrder];
  int64_t acc = 1;
  for (int m = X.n - 1; m >= 0; --m) { std_stride[m] = acc; acc *= X.dims[m]; }
  const int64_t blk = acc;
  // weight of mode m's sector in the block index: |G|^(N-2-m) blocks; the last
  // mode's sector is not stored and contributes nothing.
  int64_t wsec[kMaxOrder];
  int64_t w = blk;
  for (int m = X.n - 1; m >= 0; --m) {
    if (m == X.n - 1) { wsec[m] = 0; continue; }
    wsec[m] = w;
    w *= X.hs[m];
  }
  o.gpow = 1;
  for (int i = 0; i + 1 < o.grp.count; ++i) o.gpow *= o.grp.rad[i];
  o.n_inner = 1;
  for (int i = 0; i < o.grp.count; ++i) {
    const int m = o.grp.pos[i];
    o.dim[i] = X.dims[m];
    o.stride[i] = std_stride[m];
    o.weight[i] = wsec[m];
    o.n_inner *= X.dims[m];
  }
  // complex operands: offsets in reals; a column table lists (re, im) of each column
  o.scale = p.cplx ? 2 : 1;
  o.pairs = p.cplx && !rows ? 1 : 0;
  o.count = o.gpow * o.n_inner * (o.pairs ? 2 : 1);
  return o;
}

OffsetParams affine_offsets(const Plan& p, int64_t count, int64_t per_q, int64_t step) {
  OffsetParams o;
  std::memset(&o, 0, sizeof o);
  o.g = p.g;
  o.count = count;
  o.affine = 1;
  o.aff_q = per_q;
  o.aff_i = step;
  return o;
}

XformParams make_xform(const Plan& p, int operand, bool to_aligned, int in_bytes, int out_bytes,
                       bool out_is_split, bool slice_only) {
  XformParams x;
  std::memset(&x, 0, sizeof x);     // chg (charge tables) stays nullptr until launch
  x.g = p.g;
  const OperandDesc& X = operand == 0 ? p.U : operand == 1 ? p.V : p.W;
  x.order = X.n;

  // Sector groups: rows (I for U and W, K for V), columns (K for U, J for V and W).
  SectorGroup& R = x.row;
  SectorGroup& C = x.col;
  const int G = p.g.size;
  sector_groups(p, operand, &R, &C);
  x.gpow_row = 1;
  for (int i = 0; i + 1 < R.count; ++i) x.gpow_row *= R.rad[i];
  x.gpow_col = 1;
  for (int i = 0; i + 1 < C.count; ++i) x.gpow_col *= C.rad[i];
  for (int m = 0; m < X.n; ++m) x.hs[m] = X.hs[m];
  // The contraction's workspace copy holds the live slices (q0 + q_step j) in
  // order; a whole form (standalone transforms) holds all |G|, of which only
  // q_pin is moved where one of the form's own deltas has an empty sum.
  int64_t nslices = G;
  x.q0 = 0; x.q_step = 1; x.q_full = 1;
  if (slice_only) {
    x.q0 = p.q0; x.q_step = p.q_step; x.q_full = 0;
    nslices = p.nq;
  } else if (pinned_form(p, operand)) {
    x.q0 = p.q_pin;
    nslices = 1;
  }
  x.nblocks = x.gpow_row * x.gpow_col * nslices;
  // Complex operands move as reals: each element is a (re, im) pair, one more
  // in-block dim (std stride 1) that sits innermost among the aligned columns;
  // V's complex rows go to every other real row (the odd ones are filled from
  // them: the real representation of C).
  const int cm = p.cplx ? 2 : 1;
  const int row_mult = p.cplx && operand == 1 ? 2 : 1;
  x.blk_elems = cm;
  for (int m = 0; m < X.n; ++m) x.blk_elems *= X.dims[m];
  int64_t nR = 1, nC = 1;
  for (int i = 0; i < R.count; ++i) nR *= X.dims[R.pos[i]];
  for (int i = 0; i < C.count; ++i) nC *= X.dims[C.pos[i]];
  const int64_t rows_tot = x.gpow_row * nR * row_mult, cols_tot = x.gpow_col * nC * cm;
  const AlignedLayout lay = aligned_layout(p.compute, operand);
  // the contraction's split-bf16 planes: K (U's columns, V's rows) at pitch kpad
  const bool pad = slice_only && p.compute == SYMT_COMPUTE_BF16X3 && operand < 2 && p.kpad != p.gk;
  const int64_t rows_pitch = pad && operand == 1 ? p.kpad : rows_tot;
  const int64_t cols_pitch = pad && operand == 0 ? p.kpad : cols_tot;
  x.q_stride = rows_pitch * cols_pitch;
  x.plane = (x.q_full ? static_cast<int64_t>(G) : nslices) * x.q_stride;
  // the contraction's planes interleaved by K-steps (K fastest in both operands'
  // planes, its pitch a multiple of 32)
  x.il = out_is_split && slice_only && operand < 2 && p.bf16_il ? 1 : 0;
  if (x.il) x.plane = 32;
  const int64_t row_unit = lay == kRowMajor ? cols_pitch : 1;   // aligned stride of one real row
  const int64_t col_unit = lay == kRowMajor ? 1 : rows_pitch;   // aligned stride of one real column
  x.rs_stride = nR * row_mult * row_unit;
  x.cs_stride = nC * cm * col_unit;
  x.to_aligned = to_aligned ? 1 : 0;

  // Inner dims in aligned order with both strides (in reals).
  int64_t std_stride[kMaxOrder];
  {
    int64_t acc = cm;
    for (int m = X.n - 1; m >= 0; --m) { std_stride[m] = acc; acc *= X.dims[m]; }
  }
  int nd = 0;
  int64_t size[kMaxDims], s_std[kMaxDims], s_al[kMaxDims];
  {
    int64_t acc = row_mult;
    int64_t tmp_al[kMaxOrder];
    for (int i = R.count - 1; i >= 0; --i) { tmp_al[i] = acc * row_unit; acc *= X.dims[R.pos[i]]; }
    for (int i = 0; i < R.count; ++i) {
      size[nd] = X.dims[R.pos[i]]; s_std[nd] = std_stride[R.pos[i]]; s_al[nd] = tmp_al[i]; ++nd;
    }
    acc = cm;
    for (int i = C.count - 1; i >= 0; --i) { tmp_al[i] = acc * col_unit; acc *= X.dims[C.pos[i]]; }
    for (int i = 0; i < C.count; ++i) {
      size[nd] = X.dims[C.pos[i]]; s_std[nd] = std_stride[C.pos[i]]; s_al[nd] = tmp_al[i]; ++nd;
    }
    if (p.cplx) { size[nd] = 2; s_std[nd] = 1; s_al[nd] = col_unit; ++nd; }
  }
  // Drop unit dims, then merge neighbours that nest the same way in both layouts.
  int md = 0;
  int64_t msize[kMaxDims], mstd[kMaxDims], mal[kMaxDims];
  for (int d = 0; d < nd; ++d) {
    if (size[d] == 1) continue;
    if (md > 0 && mstd[md - 1] == s_std[d] * size[d] && mal[md - 1] == s_al[d] * size[d]) {
      msize[md - 1] *= size[d];
      mstd[md - 1] = s_std[d];
      mal[md - 1] = s_al[d];
      continue;
    }
    msize[md] = size[d]; mstd[md] = s_std[d]; mal[md] = s_al[d]; ++md;
  }
  if (md == 0) { msize[0] = 1; mstd[0] = 1; mal[0] = 1; md = 1; }
  const int64_t* ss = to_aligned ? mstd : mal;
  const int64_t* ds = to_aligned ? mal : mstd;

  // Copy mode when one dim is the fastest in both layouts, else tiled transpose.
  int run = -1;
  for (int d = 0; d < md; ++d)
    if (ss[d] == 1 && ds[d] == 1) run = d;
  int a = 0, b = 0;
  for (int d = 1; d < md; ++d) {
    if (ss[d] < ss[a]) a = d;
    if (ds[d] < ds[b]) b = d;
  }
  if (run < 0 && a == b) run = a;
  x.mode = run >= 0 ? 0 : 1;
  x.tr_write = 0;
  if (run >= 0 && md > 1 && msize[run] < 16) {
    // A short common run (under 16 elements): the tiled transpose with its A side
    // (source-fastest dims, 64 elements) written in destination order moves
    // longer contiguous pieces where the A side nests in the destination too
    // (a source [A][S][B] into a destination [S][A][B]: runs of A x B, not B).
    int by2[kMaxDims];
    for (int d = 0; d < md; ++d) by2[d] = d;
    std::sort(by2, by2 + md, [&](int l, int r) { return ss[l] < ss[r]; });
    int64_t rng[kMaxDims] = {}, pa = 1;
    int na = 0;
    for (int i = 0; i < md && pa < 64; ++i) {
      const int d = by2[i];
      rng[d] = std::min<int64_t>(msize[d], (64 + pa - 1) / pa);
      pa *= msize[d];
      ++na;
    }
    std::sort(by2, by2 + md, [&](int l, int r) { return ds[l] < ds[r]; });
    int64_t wrun = 1;
    for (int i = 0; i < md; ++i) {
      const int d = by2[i];
      if (rng[d] == 0 || ds[d] != wrun) break;
      wrun *= rng[d];
      if (rng[d] < msize[d]) break;
    }
    if (na < md && wrun >= 16 && wrun >= 2 * msize[run]) {
      x.mode = 1;
      x.tr_write = 1;
      run = -1;
    }
  }
  bool in_tile[kMaxDims] = {};
  x.na = x.nb = 0;
  x.run = run;
  if (x.mode == 0) {
    in_tile[run] = true;
    x.run_len = msize[run];
    x.run_ss = ss[run];
    x.run_ds = ds[run];
  } else {
    // A: dims by increasing source stride until 64 elements (reads coalesce
    // along it); B: the remaining dims by increasing destination stride until
    // 64 elements (writes coalesce along it).  Tiny dims are merged this way
    // so that one 64 x 64 tile stays full whatever the in-block shape.
    int by[kMaxDims];
    for (int d = 0; d < md; ++d) by[d] = d;
    std::sort(by, by + md, [&](int l, int r) { return ss[l] < ss[r]; });
    int64_t pa = 1;
    for (int i = 0; i < md && pa < 64; ++i) {
      const int d = by[i];
      x.asize[x.na] = msize[d]; x.ass[x.na] = ss[d]; x.ads[x.na] = ds[d]; ++x.na;
      pa *= msize[d];
      in_tile[d] = true;
    }
    std::sort(by, by + md, [&](int l, int r) { return ds[l] < ds[r]; });
    int64_t pb = 1;
    for (int i = 0; i < md && pb < 64; ++i) {
      const int d = by[i];
      if (in_tile[d]) continue;
      x.tsize[x.nb] = msize[d]; x.tss[x.nb] = ss[d]; x.tds[x.nb] = ds[d]; ++x.nb;
      pb *= msize[d];
      in_tile[d] = true;
    }
    if (x.nb == 0 && x.na > 1) {
      // Every dim went to A: give its slowest one to B so both sides stay parallel.
      --x.na;
      x.tsize[0] = x.asize[x.na]; x.tss[0] = x.ass[x.na]; x.tds[0] = x.ads[x.na]; x.nb = 1;
      pb = x.tsize[0];
      pa = 1;
      for (int i = 0; i < x.na; ++i) pa *= x.asize[i];
    }
    x.run_len = pa;
    x.t_len = pb;
  }
  // Batch dims: the rest, ordered so that the last one has the smallest dst stride.
  int order_idx[kMaxDims];
  int nb = 0;
  for (int d = 0; d < md; ++d)
    if (!in_tile[d]) order_idx[nb++] = d;
  std::sort(order_idx, order_idx + nb, [&](int l, int r) { return ds[l] > ds[r]; });
  x.nbatch = nb;
  x.rows = 1;
  for (int i = 0; i < nb; ++i) {
    const int d = order_idx[i];
    x.bsize[i] = msize[d];
    x.bss[i] = ss[d];
    x.bds[i] = ds[d];
    x.rows *= msize[d];
  }

  if (x.mode == 0) {
    // Vector width: 16-byte accesses where every offset stays a multiple of it.
    int vec = 1;
    if (x.run_ss == 1 && x.run_ds == 1) {
      const int out_unit = out_is_split ? 2 : out_bytes;
      for (int cand : {4, 2}) {
        if (cand * in_bytes > 16 || cand * out_unit > 16) continue;
        bool ok = x.run_len % cand == 0 && x.blk_elems % cand == 0 && x.q_stride % cand == 0 &&
                  x.rs_stride % cand == 0 && x.cs_stride % cand == 0 && x.plane % cand == 0;
        for (int i = 0; i < nb && ok; ++i) ok = x.bss[i] % cand == 0 && x.bds[i] % cand == 0;
        if (ok) { vec = cand; break; }
      }
    }
    x.vec = vec;
    const int64_t vecs = (x.run_len + vec - 1) / vec;
    int lanes = 1, lg = 0;
    while (lanes < 64 && lanes < vecs) { lanes *= 2; ++lg; }
    x.lanes_per_row = lanes;
    x.lanes_log2 = lg;
    // Long runs are cut into chunks of 8192 elements (a multiple of every
    // vector width) so that a block with few rows still spreads over many
    // workgroups (a whole matrix block can be a single run).
    x.run_chunk = x.run_len > 16384 ? 8192 : std::max<int64_t>(x.run_len, 1);
    x.run_tiles = (x.run_len + x.run_chunk - 1) / x.run_chunk;
    // rows per workgroup: about 64 KB of source each (short runs take many rows,
    // moved 1024 at a time), so the per-workgroup block arithmetic stays small
    int64_t rpt = std::max<int64_t>(1, 65536 / std::max<int64_t>(1, x.run_chunk * in_bytes));
    rpt = std::max<int64_t>(rpt, 256 / lanes);
    rpt = std::min<int64_t>(rpt, 4096);
    rpt = std::min<int64_t>(rpt, x.rows);
    // ... but keep at least 8192 workgroups (32 per compute unit) where the rows allow
    const int64_t floor_rpt = std::max<int64_t>(1, 256 / lanes);
    while (rpt > floor_rpt && rpt > 256 && x.nblocks * ((x.rows + rpt - 1) / rpt) * x.run_tiles < 8192) rpt /= 2;
    x.rows_per_tile = std::max<int64_t>(rpt, 1);
    x.tiles_per_block = (x.rows + x.rows_per_tile - 1) / x.rows_per_tile * x.run_tiles;
  } else {
    x.vec = 1;
    x.tiles_run = static_cast<int32_t>((x.run_len + 63) / 64);
    x.tiles_t = static_cast<int32_t>((x.t_len + 63) / 64);
    x.rows_per_tile = 1;
    x.tiles_per_block = x.rows * x.tiles_run * x.tiles_t;
  }
  return x;
}

}  // namespace symt

// Launch-time decision service: the driver program's run-time role, gfx950 host side.
//
// Paper: section "KLARAPTOR: A Dynamic Optimization tool for CUDA" - at run time, when a kernel
// is about to be launched, its data parameters are known; the rational program is evaluated at
// them for the admissible launch configurations, the best one is used, and the decisions are
// kept in a history so that a later launch with the same data parameters is answered from it;
// section "Input/Output Builder" - the driver turns the data sizes into the grid and block
// dimensions (gx, gy, gz, bx, by, bz) of the launch; section "Annotating the source code" - the
// user's constraints on the launch parameters are Python-syntax expressions (for example
// bx < N and bx * by <= 1024).
//
// A service holds host copies of the programs' descriptors and configurations, per-program
// compiled constraints, and the decision history (a hash map from (program, data size) to the
// decision).  A decision request for a list of data sizes answers the sizes found in the
// history at once and evaluates the others in one klr_eval_argmin call over a one-program batch
// in the caller's device workspace; with constraints, the full cost row of each of those sizes
// is copied back and the argmin is taken on the host over the configurations the constraints
// admit (strict "<" in configuration order, as on the device).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.hpp"

namespace klr {
namespace {

// ---- constraint expressions ------------------------------------------------------------------
// Python expression subset: or / and / not, chained comparisons (< <= > >= == !=), + - * / // %
// **, unary + -, parentheses, numbers, True / False, min / max / abs, and the names N (data
// size; also n, D0), bx by bz (launch parameters 0..2; also L0 L1 L2), L3, and T (the product of
// the launch parameters).  Values are doubles (exact for the integer arithmetic of launch
// parameters below 2^53); / is true division, // and % floor like Python's, and / or return
// the deciding operand as Python's do; a division by zero makes the constraint false at that
// point, as Python's exception would reject it.  At most 60 values may be pending on the
// evaluation stack.
enum Op : uint8_t {
  kConst, kVar, kAdd, kSub, kMul, kDiv, kFloorDiv, kMod, kPow, kNeg, kNot, kLt, kLe, kGt, kGe, kEq, kNe,
  kMin, kMax, kAbs,
  kOrJump,        // top true: jump to var keeping it (a or b = a); else pop and go on to b
  kAndJump        // top false: jump keeping it (a and b = a); else pop and go on to b
};
struct Ins {
  Op op;
  int32_t var;
  double val;
};
enum Var { kVN = 0, kVL0 = 1, kVL1, kVL2, kVL3, kVT, kNumVars };

struct Parser {
  const char* s;
  size_t i = 0;
  std::vector<Ins>* out;
  std::string err;

  void skip() { while (s[i] && std::isspace((unsigned char)s[i])) ++i; }
  bool word(const char* w) {
    skip();
    const size_t n = std::strlen(w);
    if (std::strncmp(s + i, w, n) != 0) return false;
    const char c = s[i + n];
    if (std::isalnum((unsigned char)c) || c == '_') return false;
    i += n;
    return true;
  }
  bool tok(const char* t) {
    skip();
    const size_t n = std::strlen(t);
    if (std::strncmp(s + i, t, n) != 0) return false;
    i += n;
    return true;
  }
  bool fail(const std::string& m) {
    if (err.empty()) err = m + " at offset " + std::to_string(i);
    return false;
  }
  void emit(Op op, int32_t var = 0, double val = 0.0) { out->push_back(Ins{op, var, val}); }

  bool expr() { return or_expr(); }
  // a or b / a and b evaluate b only when a does not decide, as Python does (so a division by
  // zero in an operand that is never reached does not reject the point)
  bool or_expr() {
    if (!and_expr()) return false;
    while (word("or")) {
      const size_t j = out->size();
      emit(kOrJump);
      if (!and_expr()) return false;
      (*out)[j].var = (int32_t)out->size();
    }
    return true;
  }
  bool and_expr() {
    if (!not_expr()) return false;
    while (word("and")) {
      const size_t j = out->size();
      emit(kAndJump);
      if (!not_expr()) return false;
      (*out)[j].var = (int32_t)out->size();
    }
    return true;
  }
  bool not_expr() {
    if (word("not")) {
      if (!not_expr()) return false;
      emit(kNot);
      return true;
    }
    return comparison();
  }
  bool cmp_op(Op* op) {
    skip();
    if (tok("<=")) { *op = kLe; return true; }
    if (tok(">=")) { *op = kGe; return true; }
    if (tok("==")) { *op = kEq; return true; }
    if (tok("!=")) { *op = kNe; return true; }
    if (s[i] == '<') { ++i; *op = kLt; return true; }
    if (s[i] == '>') { ++i; *op = kGt; return true; }
    return false;
  }
  // a < b < c is (a < b) and (b < c), with c not evaluated when a < b is false (Python's
  // chaining); the middle operand's code is emitted twice (expressions have no side effects)
  bool comparison() {
    size_t prev0 = out->size();
    if (!sum()) return false;
    std::vector<Ins> prev(out->begin() + (long)prev0, out->end());
    std::vector<size_t> jumps;
    Op op;
    int links = 0;
    while (cmp_op(&op)) {
      if (links > 0) {
        jumps.push_back(out->size());
        emit(kAndJump);
        // the copy moves: jump targets inside it (absolute positions) move with it
        const int32_t shift = (int32_t)out->size() - (int32_t)prev0;
        for (Ins x : prev) {
          if (x.op == kOrJump || x.op == kAndJump) x.var += shift;
          out->push_back(x);
        }
      }
      const size_t b0 = out->size();
      if (!sum()) return false;
      std::vector<Ins> cur(out->begin() + (long)b0, out->end());
      emit(op);
      prev.swap(cur);
      prev0 = b0;
      ++links;
    }
    for (size_t j : jumps) (*out)[j].var = (int32_t)out->size();
    return true;
  }
  bool sum() {
    if (!term()) return false;
    for (;;) {
      skip();
      if (s[i] == '+') { ++i; if (!term()) return false; emit(kAdd); }
      else if (s[i] == '-') { ++i; if (!term()) return false; emit(kSub); }
      else return true;
    }
  }
  bool term() {
    if (!factor()) return false;
    for (;;) {
      skip();
      if (tok("//")) { if (!factor()) return false; emit(kFloorDiv); }
      else if (s[i] == '*' && s[i + 1] != '*') { ++i; if (!factor()) return false; emit(kMul); }
      else if (s[i] == '/') { ++i; if (!factor()) return false; emit(kDiv); }
      else if (s[i] == '%') { ++i; if (!factor()) return false; emit(kMod); }
      else return true;
    }
  }
  bool factor() {
    skip();
    if (s[i] == '-') { ++i; if (!factor()) return false; emit(kNeg); return true; }
    if (s[i] == '+') { ++i; return factor(); }
    return power();
  }
  bool power() {
    if (!atom()) return false;
    if (tok("**")) {
      if (!factor()) return false;     // right-associative, binds tighter than unary minus on its left
      emit(kPow);
    }
    return true;
  }
  bool atom() {
    skip();
    const char c = s[i];
    if (c == '(') {
      ++i;
      if (!expr()) return false;
      if (!tok(")")) return fail("expected ')'");
      return true;
    }
    if (std::isdigit((unsigned char)c) || (c == '.' && std::isdigit((unsigned char)s[i + 1]))) {
      char* end = nullptr;
      const double v = std::strtod(s + i, &end);
      if (end == s + i) return fail("bad number");
      i = (size_t)(end - s);
      emit(kConst, 0, v);
      return true;
    }
    if (std::isalpha((unsigned char)c) || c == '_') {
      size_t j = i;
      while (std::isalnum((unsigned char)s[j]) || s[j] == '_') ++j;
      const std::string name(s + i, j - i);
      i = j;
      if (name == "True") { emit(kConst, 0, 1.0); return true; }
      if (name == "False") { emit(kConst, 0, 0.0); return true; }
      if (name == "min" || name == "max" || name == "abs") {
        if (!tok("(")) return fail("expected '(' after " + name);
        int args = 0;
        if (!tok(")")) {
          for (;;) {
            if (!expr()) return false;
            ++args;
            if (args > 1 && name != "abs") emit(name == "min" ? kMin : kMax);
            if (tok(")")) break;
            if (!tok(",")) return fail("expected ',' or ')'");
          }
        }
        if (name == "abs") {
          if (args != 1) return fail("abs takes one argument");
          emit(kAbs);
        } else if (args < 2) {
          return fail(name + " needs at least two arguments");
        }
        return true;
      }
      int var = -1;
      if (name == "N" || name == "n" || name == "D0") var = kVN;
      else if (name == "bx" || name == "L0") var = kVL0;
      else if (name == "by" || name == "L1") var = kVL1;
      else if (name == "bz" || name == "L2") var = kVL2;
      else if (name == "L3") var = kVL3;
      else if (name == "T") var = kVT;
      if (var < 0) return fail("unknown name '" + name + "'");
      emit(kVar, var);
      return true;
    }
    return fail(c ? std::string("unexpected '") + c + "'" : std::string("unexpected end"));
  }
};

bool compile(const char* src, std::vector<Ins>& code, std::string& err) {
  code.clear();
  Parser p{src, 0, &code, {}};
  if (!p.expr()) { err = p.err; return false; }
  p.skip();
  if (src[p.i] != 0) { err = "trailing text at offset " + std::to_string(p.i); return false; }
  // the program must leave exactly one value
  int depth = 0, most = 0;
  for (const Ins& x : code) {
    if (x.op == kConst || x.op == kVar) ++depth;
    else if (x.op == kNeg || x.op == kNot || x.op == kAbs) { if (depth < 1) { err = "malformed"; return false; } }
    else if (x.op == kOrJump || x.op == kAndJump) { if (depth < 1) { err = "malformed"; return false; } --depth; }
    else { if (depth < 2) { err = "malformed"; return false; } --depth; }
    most = depth > most ? depth : most;
  }
  if (depth != 1) { err = "malformed"; return false; }
  if (most > 60) { err = "expression nested too deeply"; return false; }
  return true;
}

// Truth of a compiled constraint at one point; false where a division by zero occurs.
bool holds(const std::vector<Ins>& code, const double* vars) {
  double st[64];
  int sp = 0;
  for (size_t pc = 0; pc < code.size(); ++pc) {
    const Ins& x = code[pc];
    if (sp >= 62) return false;
    switch (x.op) {
      case kOrJump:
      case kAndJump: {
        const bool truth = st[sp - 1] != 0.0;           // NaN is true, as in Python
        if (truth == (x.op == kOrJump)) pc = (size_t)x.var - 1;
        else --sp;
        break;
      }
      case kConst: st[sp++] = x.val; break;
      case kVar: st[sp++] = vars[x.var]; break;
      case kNeg: st[sp - 1] = -st[sp - 1]; break;
      case kNot: st[sp - 1] = st[sp - 1] == 0.0 ? 1.0 : 0.0; break;
      case kAbs: st[sp - 1] = std::fabs(st[sp - 1]); break;
      default: {
        const double b = st[--sp], a = st[sp - 1];
        double r = 0.0;
        switch (x.op) {
          case kAdd: r = a + b; break;
          case kSub: r = a - b; break;
          case kMul: r = a * b; break;
          case kDiv: if (b == 0.0) return false; r = a / b; break;
          case kFloorDiv: if (b == 0.0) return false; r = std::floor(a / b); break;
          case kMod: if (b == 0.0) return false; r = a - b * std::floor(a / b); break;
          case kPow: r = std::pow(a, b); break;
          case kLt: r = a < b; break;
          case kLe: r = a <= b; break;
          case kGt: r = a > b; break;
          case kGe: r = a >= b; break;
          case kEq: r = a == b; break;
          case kNe: r = a != b; break;
          case kMin: r = b < a ? b : a; break;
          case kMax: r = b > a ? b : a; break;
          default: return false;
        }
        st[sp - 1] = r;
      }
    }
  }
  return sp == 1 && st[0] != 0.0;                     // NaN is true, as in Python
}

void point_vars(int32_t N, const int32_t* L, int v_launch, double* vars) {
  vars[kVN] = (double)N;
  double T = 1.0;
  for (int k = 0; k < 4; ++k) {
    const double x = k < v_launch ? (double)L[k] : 1.0;
    vars[kVL0 + k] = x;
    T *= x;
  }
  vars[kVT] = T;
}

}  // namespace
}  // namespace klr

struct klr_service_s {
  klr_handle h = nullptr;
  std::vector<klr_program> progs;             // host copies
  std::vector<int32_t> cfgs;
  klr_hw hw{};
  const klr_fit_desc* desc = nullptr;         // device
  int32_t n_fits = 0;
  const uint8_t* exps = nullptr;              // device
  int32_t n_exp_rows = 0;
  const double* coef = nullptr;               // device
  int64_t coef_len = 0;
  const int32_t* cfgs_dev = nullptr;          // device
  int32_t max_cfg = 0, max_batch = 0;
  char* ws = nullptr;                          // device workspace
  size_t ws_bytes = 0;
  std::vector<std::vector<std::vector<klr::Ins>>> constraints;   // per program, a conjunction
  std::unordered_map<uint64_t, klr_launch> history;
  int64_t max_history = 1 << 20;
  int64_t hits = 0, misses = 0, evaluations = 0;
};

namespace klr {
namespace {

// Device workspace layout of a service: program descriptor, queries, argmin, best cost, cost
// rows (max_batch x max_cfg), program status, then the evaluation workspace of one program.
struct SvcLayout {
  size_t prog, q, am, bc, costs, st, ews, total;
};
SvcLayout svc_layout(int32_t max_cfg, int32_t max_batch) {
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  SvcLayout L{};
  size_t o = 0;
  L.prog = o; o += al(sizeof(klr_program));
  L.q = o; o += al((size_t)max_batch * 4);
  L.am = o; o += al((size_t)max_batch * 4);
  L.bc = o; o += al((size_t)max_batch * 4);
  L.costs = o; o += al((size_t)max_batch * (size_t)max_cfg * 4);
  L.st = o; o += al(4);
  L.ews = o; o += al(eval_workspace_bytes(1, max_cfg));
  L.total = o;
  return L;
}

klr_launch make_launch(const klr_service_s& s, const klr_program& P, int32_t N, int32_t c, float cost) {
  klr_launch r{};
  r.config = c;
  r.cost = cost;
  if (c < 0) return r;
  const int32_t* L = s.cfgs.data() + P.cfg0 + (int64_t)c * P.v_launch;
  r.bx = L[0];
  r.by = P.v_launch > 1 ? L[1] : 1;
  r.bz = P.v_launch > 2 ? L[2] : 1;
  int64_t T = 1;
  for (int k = 0; k < P.v_launch; ++k) T *= L[k];
  const int64_t n = N > 0 ? N : 1;
  if (P.grid_kind == KLR_GRID_2D && P.v_launch >= 2) {
    r.gx = (int32_t)((n + L[0] - 1) / L[0]);
    r.gy = (int32_t)((n + L[1] - 1) / L[1]);
  } else {
    r.gx = (int32_t)((n + T - 1) / T);
    r.gy = 1;
  }
  r.gz = 1;
  return r;
}

}  // namespace
}  // namespace klr

using klr::fail;

extern "C" {

size_t klr_service_workspace(int32_t max_cfg, int32_t max_batch) {
  if (max_cfg < 1 || max_batch < 1) return 0;
  return klr::svc_layout(max_cfg, max_batch).total;
}

klr_status klr_service_create(klr_handle h, klr_service* out, const klr_program* progs, int32_t n_progs,
                              const klr_hw* hw, const klr_fit_desc* desc, int32_t n_fits, const uint8_t* exps,
                              int32_t n_exp_rows, const double* coef, int64_t coef_len, const int32_t* cfgs_host,
                              const int32_t* cfgs_dev, int64_t cfgs_len, int32_t max_batch, void* ws,
                              size_t ws_bytes) {
  if (!h || !out) return KLR_E_INVALID;
  *out = nullptr;
  h->err.clear();
  if (!progs || n_progs < 1 || !hw || !desc || !exps || !coef || !cfgs_host || !cfgs_dev || cfgs_len < 0 ||
      max_batch < 1 || n_fits < 0 || n_exp_rows < 0 || coef_len < 0)
    return fail(h, KLR_E_INVALID, "klr_service_create: bad arguments");
  int32_t max_cfg = 1;
  for (int32_t p = 0; p < n_progs; ++p) {
    const klr_program& P = progs[p];
    if (P.v_launch < 1 || P.v_launch > KLR_MAX_LAUNCH || P.n_cfg < 0 || P.cfg0 < 0 ||
        P.cfg0 + (int64_t)P.n_cfg * P.v_launch > cfgs_len)
      return fail(h, KLR_E_INVALID, "klr_service_create: program " + std::to_string(p) + " out of range");
    if (P.n_cfg > max_cfg) max_cfg = P.n_cfg;
  }
  if (max_cfg > 65536) return fail(h, KLR_E_UNSUPPORTED, "klr_service_create: more than 65536 configurations");
  const klr::SvcLayout L = klr::svc_layout(max_cfg, max_batch);
  if (!ws || ws_bytes < L.total)
    return fail(h, KLR_E_WORKSPACE, "klr_service_create: workspace too small: need " + std::to_string(L.total));
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(h, KLR_E_INVALID, "workspace must be 256-byte aligned");
  klr_service s = new (std::nothrow) klr_service_s;
  if (!s) return fail(h, KLR_E_HIP, "out of host memory");
  s->h = h;
  s->progs.assign(progs, progs + n_progs);
  s->cfgs.assign(cfgs_host, cfgs_host + cfgs_len);
  s->hw = *hw;
  s->desc = desc;
  s->n_fits = n_fits;
  s->exps = exps;
  s->n_exp_rows = n_exp_rows;
  s->coef = coef;
  s->coef_len = coef_len;
  s->cfgs_dev = cfgs_dev;
  s->max_cfg = max_cfg;
  s->max_batch = max_batch;
  s->ws = reinterpret_cast<char*>(ws);
  s->ws_bytes = ws_bytes;
  s->constraints.resize((size_t)n_progs);
  *out = s;
  return KLR_OK;
}

void klr_service_destroy(klr_service s) { delete s; }

klr_status klr_service_add_constraint(klr_service s, int32_t prog, const char* expr) {
  if (!s) return KLR_E_INVALID;
  klr_handle h = s->h;
  h->err.clear();
  if (!expr || prog < -1 || prog >= (int32_t)s->progs.size())
    return fail(h, KLR_E_INVALID, "klr_service_add_constraint: bad program or expression");
  std::vector<klr::Ins> code;
  std::string err;
  if (!klr::compile(expr, code, err)) return fail(h, KLR_E_INVALID, "constraint '" + std::string(expr) + "': " + err);
  for (int32_t p = 0; p < (int32_t)s->progs.size(); ++p)
    if (prog < 0 || p == prog) s->constraints[(size_t)p].push_back(code);
  // earlier decisions no longer hold
  s->history.clear();
  return KLR_OK;
}

klr_status klr_service_decide(klr_service s, int32_t prog, const int32_t* N, int32_t n, klr_launch* out,
                              void* stream) {
  if (!s) return KLR_E_INVALID;
  klr_handle h = s->h;
  h->err.clear();
  if (prog < 0 || prog >= (int32_t)s->progs.size() || n < 0 || (n > 0 && (!N || !out)))
    return fail(h, KLR_E_INVALID, "klr_service_decide: bad arguments");
  const klr_program& P0 = s->progs[(size_t)prog];
  const bool constrained = !s->constraints[(size_t)prog].empty();
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const klr::SvcLayout L = klr::svc_layout(s->max_cfg, s->max_batch);
  // answer from the history; collect the distinct missing sizes
  std::vector<int32_t> miss;
  std::unordered_map<int32_t, int32_t> miss_pos;
  for (int32_t i = 0; i < n; ++i) {
    const uint64_t key = ((uint64_t)(uint32_t)prog << 32) | (uint32_t)N[i];
    auto it = s->history.find(key);
    if (it != s->history.end()) { out[i] = it->second; ++s->hits; continue; }
    ++s->misses;
    if (miss_pos.find(N[i]) == miss_pos.end()) { miss_pos[N[i]] = (int32_t)miss.size(); miss.push_back(N[i]); }
  }
  std::vector<klr_launch> decided(miss.size());
  for (size_t b0 = 0; b0 < miss.size(); b0 += (size_t)s->max_batch) {
    const int32_t nb = (int32_t)std::min(miss.size() - b0, (size_t)s->max_batch);
    klr_program P = P0;
    P.q0 = 0;
    P.n_q = nb;
    P.cost0 = 0;
    hipError_t e = hipMemcpyAsync(s->ws + L.prog, &P, sizeof(P), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(s->ws + L.q, miss.data() + b0, (size_t)nb * 4, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return klr::hip_check(h, e, "klr_service_decide upload");
    float* costs = constrained ? reinterpret_cast<float*>(s->ws + L.costs) : nullptr;
    klr_status rc = klr_eval_argmin(h, reinterpret_cast<const klr_program*>(s->ws + L.prog), 1, s->max_cfg, nb,
                                    &s->hw, s->desc, s->n_fits, s->exps, s->n_exp_rows, s->coef, s->coef_len,
                                    s->cfgs_dev, (int64_t)s->cfgs.size(), reinterpret_cast<const int32_t*>(s->ws + L.q),
                                    nb, reinterpret_cast<int32_t*>(s->ws + L.am), reinterpret_cast<float*>(s->ws + L.bc),
                                    costs, costs ? (int64_t)nb * P.n_cfg : 0,
                                    reinterpret_cast<int32_t*>(s->ws + L.st), s->ws + L.ews, L.total - L.ews, stream);
    if (rc != KLR_OK) return rc;
    ++s->evaluations;
    std::vector<int32_t> am((size_t)nb), pst(1);
    std::vector<float> bc((size_t)nb), cost_rows;
    e = hipMemcpyAsync(am.data(), s->ws + L.am, (size_t)nb * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(bc.data(), s->ws + L.bc, (size_t)nb * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(pst.data(), s->ws + L.st, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && constrained) {
      cost_rows.resize((size_t)nb * P.n_cfg);
      e = hipMemcpyAsync(cost_rows.data(), costs, cost_rows.size() * 4, hipMemcpyDeviceToHost, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return klr::hip_check(h, e, "klr_service_decide download");
    if (pst[0] & KLR_PROG_BAD_DESC)
      return fail(h, KLR_E_INVALID, "klr_service_decide: program " + std::to_string(prog) + " descriptor invalid");
    for (int32_t q = 0; q < nb; ++q) {
      int32_t c = am[(size_t)q];
      float best = bc[(size_t)q];
      if (constrained) {
        // argmin over the configurations the constraints admit, strict "<" in index order
        c = -1;
        best = INFINITY;
        double vars[klr::kNumVars];
        for (int32_t k = 0; k < P.n_cfg; ++k) {
          const float v = cost_rows[(size_t)k * nb + q];      // configuration-major rows
          if (!(v < best)) continue;
          klr::point_vars(miss[b0 + q], s->cfgs.data() + P.cfg0 + (int64_t)k * P.v_launch, P.v_launch, vars);
          bool okc = true;
          for (const auto& code : s->constraints[(size_t)prog])
            if (!klr::holds(code, vars)) { okc = false; break; }
          if (okc) { best = v; c = k; }
        }
      }
      decided[b0 + q] = klr::make_launch(*s, P0, miss[b0 + q], c, best);
    }
  }
  if ((int64_t)s->history.size() + (int64_t)miss.size() > s->max_history) s->history.clear();
  for (size_t j = 0; j < miss.size(); ++j)
    s->history[((uint64_t)(uint32_t)prog << 32) | (uint32_t)miss[j]] = decided[j];
  for (int32_t i = 0; i < n; ++i) {
    auto it = miss_pos.find(N[i]);
    if (it != miss_pos.end() && s->history.count(((uint64_t)(uint32_t)prog << 32) | (uint32_t)N[i]))
      out[i] = decided[(size_t)it->second];
  }
  return KLR_OK;
}

klr_status klr_service_stats(klr_service s, int64_t* hits, int64_t* misses, int64_t* evaluations,
                             int64_t* entries) {
  if (!s) return KLR_E_INVALID;
  if (hits) *hits = s->hits;
  if (misses) *misses = s->misses;
  if (evaluations) *evaluations = s->evaluations;
  if (entries) *entries = (int64_t)s->history.size();
  return KLR_OK;
}

klr_status klr_service_set_history_limit(klr_service s, int64_t max_entries) {
  if (!s || max_entries < 0) return KLR_E_INVALID;
  s->max_history = max_entries;
  if ((int64_t)s->history.size() > max_entries) s->history.clear();
  return KLR_OK;
}

int32_t klr_constraint_check(const char* expr, int32_t N, const int32_t* L, int32_t v_launch, char* err,
                             int32_t err_len) {
  std::vector<klr::Ins> code;
  std::string e;
  if (!expr || v_launch < 0 || v_launch > KLR_MAX_LAUNCH || (v_launch > 0 && !L)) {
    if (err && err_len > 0) std::snprintf(err, (size_t)err_len, "bad arguments");
    return -1;
  }
  if (!klr::compile(expr, code, e)) {
    if (err && err_len > 0) std::snprintf(err, (size_t)err_len, "%s", e.c_str());
    return -1;
  }
  double vars[klr::kNumVars];
  klr::point_vars(N, L, v_launch, vars);
  return klr::holds(code, vars) ? 1 : 0;
}

}  // extern "C"

// Instrumentation pass (Section 2.2): turns a structured program into the
// kernel model that the repair loop takes.
//
// Sites.  In the kernel body (function 0) an instrumented barrier -- a
// BLOCK-level barrier variable, followed by a GRID-level one when grid
// instrumentation is enabled -- is placed before every access, before every
// branch (at its entry point, outside the branch), at the head of every loop
// (first thing of each iteration) and before every call whose callee reaches
// an access.  Called functions are not instrumented inside: the site before
// the call stands for them, as in the paper's example kernel.  Every
// pre-existing barrier, wherever it is, becomes a barrier variable of its own
// level marked pre-existing, so the repair may remove it.
//
// Expansion.  Loops are unrolled and calls inlined in execution order; one
// barrier variable is one static site (or one pre-existing barrier per chain
// of call sites) and its unrolled copies are occurrences of it.  A branch
// runs its body under the conjunction of its condition (tid % m == r and
// bid % bm == br) and the enclosing one: each part is again a residue class
// (Chinese remainder theorem).
// An access word is (a*tid + b*bid + c + d*it) mod words with it the
// iteration of the innermost enclosing loop (0 outside loops).  The weight
// of a variable is gw*gb + lw^ld (Section 2.4), ld the number of loops
// around it.  Slots are numbered by first occurrence, guards by first use
// after guard 0 = {1, 0}.
#include <cstring>
#include <map>
#include <vector>

#include "common.h"

namespace rp {
namespace {

constexpr uint32_t MAX_CALL_DEPTH = 64;
constexpr uint64_t MAX_STEPS = 1ull << 24;

struct SiteKey {
  std::vector<uint64_t> path;   // (function << 32 | statement) of each call site, then the site's own
  uint32_t tag;                 // 0 block site, 1 grid site, 2 pre-existing barrier
  bool operator<(const SiteKey& o) const {
    if (path != o.path) return path < o.path;
    return tag < o.tag;
  }
};

struct Cond {                                 // a guard: thread part, block part
  rp_guard t, b;
};

struct Pass {
  const rp_program* p;
  uint8_t grid;
  uint32_t gw, lw;
  std::vector<std::vector<uint32_t>> match;   // per function: END index of each IF/LOOP
  std::vector<int8_t> reaches;                // per function: an access is reachable
  std::vector<Cond> guards;                   // output guard table
  std::vector<rp_point> points;
  std::vector<rp_slot> slots;
  std::map<SiteKey, uint32_t> slot_of;
  std::vector<uint64_t> path;
  uint64_t steps = 0;                         // statements visited, loop iterations
  int err = RP_OK;

  static uint64_t gcd(uint64_t a, uint64_t b) {
    while (b) { const uint64_t t = a % b; a = b; b = t; }
    return a;
  }

  // t = r1 (mod m1) and t = r2 (mod m2) as one residue class, or false
  static bool compose(rp_guard g1, rp_guard g2, rp_guard& out) {
    const uint64_t m1 = g1.m, m2 = g2.m;
    const uint64_t g = gcd(m1, m2);
    const int64_t diff = (int64_t)g2.r - (int64_t)g1.r;
    if (diff % (int64_t)g != 0) return false;
    const uint64_t M = m1 / g * m2;
    if (M > 0xffffffffull) return false;
    // solve m1*k = diff (mod m2): k = (diff/g) * inv(m1/g) mod (m2/g)
    const int64_t n = (int64_t)(m2 / g);
    int64_t k = 0;
    if (n > 1) {
      int64_t a = (int64_t)((m1 / g) % (uint64_t)n), b = n, x0 = 1, x1 = 0;
      while (b) {                               // extended Euclid: x0*(m1/g) = 1 (mod n)
        const int64_t q = a / b, t = a - q * b;
        a = b; b = t;
        const int64_t tx = x0 - q * x1;
        x0 = x1; x1 = tx;
      }
      const int64_t inv = ((x0 % n) + n) % n;
      const int64_t dq = (((diff / (int64_t)g) % n) + n) % n;
      k = (int64_t)(((__int128)dq * inv) % n);
    }
    const uint64_t R = (uint64_t)(((__int128)g1.r + (__int128)k * (__int128)m1) % (__int128)M);
    out.m = (uint32_t)M;
    out.r = (uint32_t)R;
    return true;
  }

  uint16_t guard_id(Cond g) {
    for (size_t i = 0; i < guards.size(); i++)
      if (guards[i].t.m == g.t.m && guards[i].t.r == g.t.r && guards[i].b.m == g.b.m &&
          guards[i].b.r == g.b.r)
        return (uint16_t)i;
    guards.push_back(g);
    return (uint16_t)(guards.size() - 1);
  }

  Cond cond_of(uint16_t g) const {
    Cond c;
    c.t = p->guards[g];
    c.b = p->block_guards ? p->block_guards[g] : rp_guard{1, 0};
    return c;
  }

  uint32_t weight(uint8_t level, uint32_t depth) {
    uint64_t w = 1;
    for (uint32_t i = 0; i < depth; i++) {
      w *= lw;
      if (w > 0xffffffffull) { err = RP_ERR_INVALID; return 1; }
    }
    w += level == RP_GRID ? (uint64_t)gw : 0;
    if (w > 0xffffffffull || w == 0) { err = RP_ERR_INVALID; return 1; }
    return (uint32_t)w;
  }

  // the model's limits, and a bound on the walk itself (empty loops)
  bool full() {
    if (points.size() > (size_t)MAX_POINTS || slots.size() > 64 || ++steps > MAX_STEPS)
      err = RP_ERR_INVALID;
    return err != RP_OK;
  }

  void barrier(uint32_t f, uint32_t s, uint32_t tag, uint8_t level, uint8_t pre, uint16_t g,
               uint32_t depth) {
    SiteKey key;
    key.path = path;
    key.path.push_back((uint64_t)f << 32 | s);
    key.tag = tag;
    auto it = slot_of.find(key);
    uint32_t slot;
    if (it == slot_of.end()) {
      slot = (uint32_t)slots.size();
      rp_slot sl;
      std::memset(&sl, 0, sizeof(sl));
      sl.level = level;
      sl.preexisting = pre;
      sl.weight = weight(level, depth);
      slots.push_back(sl);
      slot_of.emplace(std::move(key), slot);
    } else {
      slot = it->second;
    }
    rp_point pt;
    std::memset(&pt, 0, sizeof(pt));
    pt.kind = RP_BARRIER;
    pt.guard = g;
    pt.slot = (uint16_t)slot;
    points.push_back(pt);
  }

  void site(uint32_t f, uint32_t s, uint16_t g, uint32_t depth) {
    barrier(f, s, 0, RP_BLOCK, 0, g, depth);
    if (grid) barrier(f, s, 1, RP_GRID, 0, g, depth);
  }

  void expand(uint32_t f, uint32_t lo, uint32_t hi, Cond gcur, uint32_t depth, int64_t it) {
    const rp_function& fn = p->functions[f];
    int32_t gi = -1;                            // guard index, taken at first use
    auto G = [&]() -> uint16_t {
      if (gi < 0) gi = guard_id(gcur);
      return (uint16_t)gi;
    };
    for (uint32_t s = lo; s < hi && !full(); s++) {
      const rp_stmt& st = fn.stmts[s];
      switch (st.kind) {
        case RP_S_ACCESS: {
          if (f == 0) site(f, s, G(), depth);
          rp_point pt;
          std::memset(&pt, 0, sizeof(pt));
          pt.kind = RP_ACCESS;
          pt.is_write = st.is_write;
          pt.array = st.array;
          pt.guard = G();
          pt.a = st.a;
          pt.b = st.b;
          const int64_t c = (int64_t)st.c + (int64_t)st.d * it;
          if (c < INT32_MIN || c > INT32_MAX) { err = RP_ERR_INVALID; return; }
          pt.c = (int32_t)c;
          points.push_back(pt);
          break;
        }
        case RP_S_BARRIER:
          barrier(f, s, 2, st.level, 1, G(), depth);
          break;
        case RP_S_IF: {
          if (f == 0) site(f, s, G(), depth);
          Cond inner;
          const Cond c = cond_of(st.guard);
          if (!compose(gcur.t, c.t, inner.t) || !compose(gcur.b, c.b, inner.b)) {
            err = RP_ERR_INVALID;
            return;
          }
          const uint32_t end = match[f][s];
          expand(f, s + 1, end, inner, depth, it);
          s = end;
          break;
        }
        case RP_S_LOOP: {
          const uint32_t end = match[f][s];
          for (uint32_t i = 0; i < st.count && !full(); i++) {
            if (f == 0) site(f, s, G(), depth + 1);
            expand(f, s + 1, end, gcur, depth + 1, i);
          }
          s = end;
          break;
        }
        case RP_S_CALL: {
          if (f == 0 && reaches[st.count]) site(f, s, G(), depth);
          path.push_back((uint64_t)f << 32 | s);
          expand(st.count, 0, p->functions[st.count].n_stmts, gcur, depth, it);
          path.pop_back();
          break;
        }
        default:
          err = RP_ERR_INVALID;
          return;
      }
      if (err != RP_OK) return;
    }
  }

  // structure checks: balanced IF/LOOP ... END, indices in range, no
  // recursion, and which functions reach an access
  int check() {
    if (!p || p->blocks < 1 || p->threads < 1 || p->n_functions < 1 || !p->functions)
      return RP_ERR_INVALID;
    if ((p->n_arrays && !p->arrays) || (p->n_guards && !p->guards)) return RP_ERR_INVALID;
    for (uint32_t a = 0; a < p->n_arrays; a++)
      if (p->arrays[a].words < 1 || p->arrays[a].space > 1) return RP_ERR_INVALID;
    for (uint32_t g = 0; g < p->n_guards; g++) {
      if (p->guards[g].m < 1 || p->guards[g].r >= p->guards[g].m) return RP_ERR_INVALID;
      if (p->block_guards && (p->block_guards[g].m < 1 ||
                              p->block_guards[g].r >= p->block_guards[g].m))
        return RP_ERR_INVALID;
    }
    const uint32_t F = p->n_functions;
    match.assign(F, {});
    for (uint32_t f = 0; f < F; f++) {
      const rp_function& fn = p->functions[f];
      if (fn.n_stmts && !fn.stmts) return RP_ERR_INVALID;
      match[f].assign(fn.n_stmts, 0);
      std::vector<uint32_t> open;
      for (uint32_t s = 0; s < fn.n_stmts; s++) {
        const rp_stmt& st = fn.stmts[s];
        switch (st.kind) {
          case RP_S_ACCESS:
            if (st.array >= p->n_arrays || st.is_write > 1) return RP_ERR_INVALID;
            break;
          case RP_S_BARRIER:
            if (st.level > RP_GRID) return RP_ERR_INVALID;
            break;
          case RP_S_IF:
            if (st.guard >= p->n_guards) return RP_ERR_INVALID;
            open.push_back(s);
            break;
          case RP_S_LOOP:
            if (st.count < 1) return RP_ERR_INVALID;
            open.push_back(s);
            break;
          case RP_S_CALL:
            if (st.count >= F || st.count == 0) return RP_ERR_INVALID;
            break;
          case RP_S_END:
            if (open.empty()) return RP_ERR_INVALID;
            match[f][open.back()] = s;
            open.pop_back();
            break;
          default:
            return RP_ERR_INVALID;
        }
      }
      if (!open.empty()) return RP_ERR_INVALID;
    }
    // call graph: depth-first with colours; a back edge is recursion
    std::vector<int8_t> colour(F, 0);
    reaches.assign(F, 0);
    std::vector<std::pair<uint32_t, uint32_t>> stack;
    for (uint32_t root = 0; root < F; root++) {
      if (colour[root]) continue;
      stack.push_back({root, 0});
      colour[root] = 1;
      while (!stack.empty()) {
        auto& top = stack.back();
        const rp_function& fn = p->functions[top.first];
        if (top.second < fn.n_stmts) {
          const rp_stmt& st = fn.stmts[top.second++];
          if (st.kind == RP_S_ACCESS) reaches[top.first] = 1;
          if (st.kind == RP_S_CALL) {
            if (colour[st.count] == 1) return RP_ERR_INVALID;
            if (colour[st.count] == 0) {
              if (stack.size() >= MAX_CALL_DEPTH) return RP_ERR_INVALID;
              colour[st.count] = 1;
              stack.push_back({st.count, 0});
            } else if (reaches[st.count]) {
              reaches[top.first] = 1;
            }
          }
        } else {
          const uint32_t done = top.first;
          colour[done] = 2;
          stack.pop_back();
          if (!stack.empty() && reaches[done]) reaches[stack.back().first] = 1;
        }
      }
    }
    return RP_OK;
  }
};

}  // namespace
}  // namespace rp

extern "C" rp_status rp_instrument(const rp_program* prog, const rp_instrument_opts* opts,
                                   rp_guard* guards, rp_guard* block_guards, uint32_t guards_cap,
                                   uint32_t* n_guards,
                                   rp_point* points, uint32_t points_cap, uint32_t* n_points,
                                   rp_slot* slots, uint32_t slots_cap, uint32_t* n_slots) {
  using namespace rp;
  if (!n_guards || !n_points || !n_slots) return RP_ERR_INVALID;
  Pass ps;
  ps.p = prog;
  ps.grid = opts ? opts->grid : 1;
  ps.gw = opts ? opts->gw : 12;
  ps.lw = opts ? opts->lw : 10;
  if (ps.grid > 1 || ps.lw < 1) return RP_ERR_INVALID;
  int st = ps.check();
  if (st != RP_OK) return (rp_status)st;
  const Cond all{rp_guard{1, 0}, rp_guard{1, 0}};
  ps.guards.push_back(all);
  ps.expand(0, 0, prog->functions[0].n_stmts, all, 0, 0);
  if (ps.points.size() > (size_t)MAX_POINTS || ps.slots.size() > 64) ps.err = RP_ERR_INVALID;
  if (ps.err != RP_OK) return (rp_status)ps.err;
  *n_guards = (uint32_t)ps.guards.size();
  *n_points = (uint32_t)ps.points.size();
  *n_slots = (uint32_t)ps.slots.size();
  if (ps.guards.size() > guards_cap || ps.points.size() > points_cap || ps.slots.size() > slots_cap)
    return RP_ERR_CAPACITY;
  if ((ps.guards.size() && (!guards || !block_guards)) || (ps.points.size() && !points) ||
      (ps.slots.size() && !slots))
    return RP_ERR_INVALID;
  for (size_t g = 0; g < ps.guards.size(); g++) {
    guards[g] = ps.guards[g].t;
    block_guards[g] = ps.guards[g].b;
  }
  std::memcpy(points, ps.points.data(), ps.points.size() * sizeof(rp_point));
  std::memcpy(slots, ps.slots.data(), ps.slots.size() * sizeof(rp_slot));
  return RP_OK;
}

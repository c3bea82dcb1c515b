/*
 * CPU oracle for the barrier-repair path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only tests/, the smoke entry point and the benchmark's CPU-baseline leg
 * load this library.  It is deliberately plain: records are materialised,
 * grouped with std::sort and compared pairwise; clauses are reduced by an
 * O(n^2) subsumption sweep; the solver enumerates assignments (or runs a
 * plain depth-first branch and bound on large components).
 *
 * Definitions followed (Joshi & Muduganti, arXiv 2011.08373):
 *   - data race: two threads touch one location, at least one writes, with
 *     no barrier in between (Section 1, Listing 1);
 *   - barrier divergence: a barrier reached by only part of a block
 *     (Section 1, Listing 2), a grid-level one by only part of the grid;
 *   - a block-level barrier orders threads of one block, a grid-level
 *     barrier orders every pair of threads (Section 1; Section 2.2);
 *   - instrumented barriers guarded by barrier variables, pre-existing
 *     barriers guarded too (Section 2.2);
 *   - race -> positive clause over the barrier variables disabled in the
 *     trace, divergence -> negative clause (Section 2.4);
 *   - Solve: weighted partial MaxSAT, hard clauses phi, soft {not b_i}
 *     weighted per Section 2.4 (weights are inputs here);
 *   - the repair loop of Alg. 1.
 *
 * Readings where the text is silent (each is listed in the design notes):
 * "between" means strictly between two program positions; an enabled
 * barrier separates every thread pair whether or not it diverges; a thread
 * never races with itself; read-read never races; each divergence clause is
 * the unit {not b_s}; ties in Solve are broken by (weight, number of enabled
 * barriers, mask as an unsigned integer); Solve returns a total assignment
 * with unconstrained variables false.
 *
 * Parity pins: every function here is exercised against worked examples of
 * the paper, closed forms and brute force in tests/test_oracle_*.py.
 */
#include "oracle.h"

#include <algorithm>
#include <atomic>
#include <cstring>
#include <thread>
#include <vector>

namespace {

typedef uint64_t u64;
typedef uint32_t u32;
typedef int64_t i64;
typedef unsigned __int128 u128;

const int ACCESS = 0, BARRIER = 1;
const int GLOBAL = 1;
const int GRID = 1;

// ---------------------------------------------------------------- validation
int validate(const or_kernel* k) {
  if (!k) return OR_ERR_INVALID;
  if (k->blocks < 1 || k->threads < 1) return OR_ERR_INVALID;
  if (k->n_slots > 64 || k->n_points > 4096) return OR_ERR_INVALID;
  if ((k->n_arrays && !k->arrays) || (k->n_guards && !k->guards) ||
      (k->n_points && !k->points) || (k->n_slots && !k->slots))
    return OR_ERR_INVALID;
  for (u32 a = 0; a < k->n_arrays; a++)
    if (k->arrays[a].words < 1 || k->arrays[a].space > 1) return OR_ERR_INVALID;
  for (u32 g = 0; g < k->n_guards; g++) {
    if (k->guards[g].m < 1 || k->guards[g].r >= k->guards[g].m) return OR_ERR_INVALID;
    if (k->block_guards &&
        (k->block_guards[g].m < 1 || k->block_guards[g].r >= k->block_guards[g].m))
      return OR_ERR_INVALID;
  }
  for (u32 s = 0; s < k->n_slots; s++)
    if (k->slots[s].level > 1 || k->slots[s].preexisting > 1 || k->slots[s].weight < 1)
      return OR_ERR_INVALID;
  std::vector<int> slot_guard(k->n_slots, -1);
  u32 next_slot = 0;
  for (u32 i = 0; i < k->n_points; i++) {
    const or_point& p = k->points[i];
    if (p.kind > 2) return OR_ERR_INVALID;
    if (p.kind == ACCESS) {
      if (p.array >= k->n_arrays || p.guard >= k->n_guards || p.is_write > 1)
        return OR_ERR_INVALID;
    } else if (p.kind == BARRIER) {
      if (p.slot >= k->n_slots || p.guard >= k->n_guards) return OR_ERR_INVALID;
      if (slot_guard[p.slot] < 0) {
        // slots are numbered by first occurrence
        if (p.slot != next_slot) return OR_ERR_INVALID;
        next_slot++;
        slot_guard[p.slot] = p.guard;
      } else if (slot_guard[p.slot] != (int)p.guard) {
        return OR_ERR_INVALID;  // all occurrences of a slot share a guard
      }
    }
  }
  if (next_slot != k->n_slots) return OR_ERR_INVALID;  // every slot occurs
  return OR_OK;
}

// ------------------------------------------------------------ model helpers
// Thread t of block blk executes point i: its guard holds for the thread
// id and, when the kernel has block conditions, for the block id.
bool active(const or_kernel* k, u32 i, u32 blk, u32 t) {
  const u32 g = k->points[i].guard;
  if (t % k->guards[g].m != k->guards[g].r) return false;
  return !k->block_guards || blk % k->block_guards[g].m == k->block_guards[g].r;
}

u64 address(const or_kernel* k, u32 i, u32 blk, u32 t) {
  const or_point& p = k->points[i];
  i64 n = (i64)k->arrays[p.array].words;
  i64 v = (i64)p.a * (i64)t + (i64)p.b * (i64)blk + (i64)p.c;
  return (u64)(((v % n) + n) % n);  // Euclidean residue in [0, n)
}

bool is_global(const or_kernel* k, u32 i) {
  return k->arrays[k->points[i].array].space == GLOBAL;
}

// An enabled barrier occurrence strictly between positions i < j.
// grid_only: only grid-level barriers count (they alone order threads of
// different blocks).
bool separated(const or_kernel* k, u64 x, u32 i, u32 j, bool grid_only) {
  for (u32 u = i + 1; u < j; u++) {
    const or_point& p = k->points[u];
    if (p.kind != BARRIER) continue;
    if (!((x >> p.slot) & 1)) continue;
    if (grid_only && k->slots[p.slot].level != GRID) continue;
    return true;
  }
  return false;
}

// Threads of block blk that execute point i.
u64 reached(const or_kernel* k, u32 i, u32 blk) {
  u64 n = 0;
  for (u32 t = 0; t < k->threads; t++)
    if (active(k, i, blk, t)) n++;
  return n;
}

// Slots that diverge when enabled.  A block-level barrier diverges when
// some block has part of its threads reaching it; a grid-level barrier must
// be reached by every thread of the grid, so it diverges when part of the
// grid reaches it (Section 1, Listing 2; Section 2.2 for the grid barrier).
// literal: count every block; otherwise the per-block count is taken once
// (it does not depend on the block) and the blocks that execute the point
// are counted from the block condition.
u64 divergent_if_enabled(const or_kernel* k, bool literal) {
  u64 mask = 0;
  for (u32 u = 0; u < k->n_points; u++) {
    const or_point& p = k->points[u];
    if (p.kind != BARRIER) continue;
    bool part_of_a_block = false;
    u64 total = 0;
    if (literal) {
      for (u32 blk = 0; blk < k->blocks; blk++) {
        const u64 n = reached(k, u, blk);
        if (n > 0 && n < k->threads) part_of_a_block = true;
        total += n;
      }
    } else {
      u64 nt = 0;
      for (u32 t = 0; t < k->threads; t++)
        if (t % k->guards[p.guard].m == k->guards[p.guard].r) nt++;
      u64 nb = 0;
      for (u32 blk = 0; blk < k->blocks; blk++)
        if (!k->block_guards || blk % k->block_guards[p.guard].m == k->block_guards[p.guard].r) nb++;
      part_of_a_block = nb > 0 && nt > 0 && nt < k->threads;
      total = nb * nt;
    }
    const bool grid = k->slots[p.slot].level == GRID;
    const bool div = grid ? total > 0 && total < (u64)k->blocks * k->threads : part_of_a_block;
    if (div) mask |= 1ull << p.slot;
  }
  return mask;
}

// Executing (block, thread) pairs of every access point: threads meeting
// the thread condition times blocks meeting the block condition.
u64 count_records(const or_kernel* k) {
  u64 n = 0;
  for (u32 i = 0; i < k->n_points; i++) {
    if (k->points[i].kind != ACCESS) continue;
    const u32 g = k->points[i].guard;
    u64 nt = 0, nb = 0;
    for (u32 t = 0; t < k->threads; t++)
      if (t % k->guards[g].m == k->guards[g].r) nt++;
    for (u32 blk = 0; blk < k->blocks; blk++)
      if (!k->block_guards || blk % k->block_guards[g].m == k->block_guards[g].r) nb++;
    n += nt * nb;
  }
  return n;
}

// Pair set as a bitmap over (level, i, j), i <= j.
struct PairSet {
  u32 P;
  std::vector<uint8_t> bits;
  explicit PairSet(u32 p) : P(p), bits(2ull * p * p, 0) {}
  void set(int lv, u32 i, u32 j) { bits[(u64)lv * P * P + (u64)i * P + j] = 1; }
  bool get(int lv, u32 i, u32 j) const { return bits[(u64)lv * P * P + (u64)i * P + j]; }
};

// -------------------------------------------- conflicts, literal definition
// Every pair of access records (i, blk, t) / (j, blk', t') is compared.
void conflicts_literal(const or_kernel* k, u64 x, bool apply_x, PairSet& out) {
  struct R { u32 i, blk, t; };
  std::vector<R> recs;
  for (u32 i = 0; i < k->n_points; i++) {
    if (k->points[i].kind != ACCESS) continue;
    for (u32 blk = 0; blk < k->blocks; blk++)
      for (u32 t = 0; t < k->threads; t++)
        if (active(k, i, blk, t)) recs.push_back({i, blk, t});
  }
  for (size_t r1 = 0; r1 < recs.size(); r1++) {
    for (size_t r2 = r1 + 1; r2 < recs.size(); r2++) {
      const R& A = recs[r1];
      const R& B = recs[r2];  // enumeration order gives A.i <= B.i
      const or_point& pa = k->points[A.i];
      const or_point& pb = k->points[B.i];
      if (pa.array != pb.array) continue;
      if (!pa.is_write && !pb.is_write) continue;          // read-read never races
      if (A.blk == B.blk && A.t == B.t) continue;           // one thread
      bool same_block = A.blk == B.blk;
      if (!same_block && !is_global(k, A.i)) continue;      // distinct shared instances
      if (address(k, A.i, A.blk, A.t) != address(k, B.i, B.blk, B.t)) continue;
      int lv = same_block ? 0 : 1;
      if (apply_x && separated(k, x, A.i, B.i, lv == 1)) continue;
      out.set(lv, A.i, B.i);
    }
  }
}

// ------------------------------------------- conflicts, grouped by location
// Same definition, evaluated per memory location: records are grouped by
// (array, block, address) for the same-block relation and by (array,
// address) for the cross-block relation; within a location every pair of
// points is examined.  Independent of any barrier assignment.

// One location of the same-block relation: its records (point i, thread t)
// sorted by (i, t), one per executing (point, thread).  Points i <= j
// conflict there when one writes and two distinct threads are involved.
struct SbRec { u32 i, t; };
void same_block_location(const or_kernel* k, const SbRec* r, size_t n, PairSet& out) {
  struct G { u32 i; u64 n; u32 t0; };
  std::vector<G> pts;
  for (size_t q = 0; q < n; q++) {
    if (pts.empty() || pts.back().i != r[q].i) pts.push_back({r[q].i, 0, r[q].t});
    pts.back().n++;  // distinct threads: one record per (point, block, thread)
  }
  for (size_t a = 0; a < pts.size(); a++) {
    const or_point& pa = k->points[pts[a].i];
    if (pa.is_write && pts[a].n >= 2) out.set(0, pts[a].i, pts[a].i);
    for (size_t b = a + 1; b < pts.size(); b++) {
      const or_point& pb = k->points[pts[b].i];
      if (!pa.is_write && !pb.is_write) continue;
      bool one_same_thread = pts[a].n == 1 && pts[b].n == 1 && pts[a].t0 == pts[b].t0;
      if (!one_same_thread) out.set(0, pts[a].i, pts[b].i);
    }
  }
}

// One location of the cross-block relation (a global array): its records
// (point i, block) sorted by (i, block), one per executing (point, block,
// thread).  Points i <= j conflict there when one writes and two distinct
// blocks are involved.
struct XbRec { u32 i, blk; };
void cross_block_location(const or_kernel* k, const XbRec* r, size_t n, PairSet& out) {
  struct G { u32 i; u64 nblk; u32 b0; };
  std::vector<G> pts;
  for (size_t q = 0; q < n; q++) {
    if (pts.empty() || pts.back().i != r[q].i) {
      pts.push_back({r[q].i, 1, r[q].blk});
    } else if (r[q].blk != r[q - 1].blk) {
      pts.back().nblk++;  // distinct blocks of this point here
    }
  }
  for (size_t a = 0; a < pts.size(); a++) {
    const or_point& pa = k->points[pts[a].i];
    if (pa.is_write && pts[a].nblk >= 2) out.set(1, pts[a].i, pts[a].i);
    for (size_t b = a + 1; b < pts.size(); b++) {
      const or_point& pb = k->points[pts[b].i];
      if (!pa.is_write && !pb.is_write) continue;
      bool one_same_block = pts[a].nblk == 1 && pts[b].nblk == 1 && pts[a].b0 == pts[b].b0;
      if (!one_same_block) out.set(1, pts[a].i, pts[b].i);
    }
  }
}

// Every location of the whole kernel at once (records of all arrays and
// blocks materialised together).
void conflicts_grouped(const or_kernel* k, PairSet& out) {
  // same block
  {
    struct R { u32 arr, blk; u64 addr; u32 i, t; };
    std::vector<R> recs;
    for (u32 i = 0; i < k->n_points; i++) {
      if (k->points[i].kind != ACCESS) continue;
      for (u32 blk = 0; blk < k->blocks; blk++)
        for (u32 t = 0; t < k->threads; t++)
          if (active(k, i, blk, t))
            recs.push_back({k->points[i].array, blk, address(k, i, blk, t), i, t});
    }
    std::sort(recs.begin(), recs.end(), [](const R& a, const R& b) {
      if (a.arr != b.arr) return a.arr < b.arr;
      if (a.blk != b.blk) return a.blk < b.blk;
      if (a.addr != b.addr) return a.addr < b.addr;
      if (a.i != b.i) return a.i < b.i;
      return a.t < b.t;
    });
    std::vector<SbRec> loc;
    size_t s = 0;
    while (s < recs.size()) {
      size_t e = s;
      while (e < recs.size() && recs[e].arr == recs[s].arr && recs[e].blk == recs[s].blk &&
             recs[e].addr == recs[s].addr)
        e++;
      loc.clear();
      for (size_t r = s; r < e; r++) loc.push_back({recs[r].i, recs[r].t});
      same_block_location(k, loc.data(), loc.size(), out);
      s = e;
    }
  }
  // different blocks (global arrays)
  {
    struct R { u32 arr; u64 addr; u32 i, blk; };
    std::vector<R> recs;
    for (u32 i = 0; i < k->n_points; i++) {
      if (k->points[i].kind != ACCESS || !is_global(k, i)) continue;
      for (u32 blk = 0; blk < k->blocks; blk++)
        for (u32 t = 0; t < k->threads; t++)
          if (active(k, i, blk, t))
            recs.push_back({k->points[i].array, address(k, i, blk, t), i, blk});
    }
    std::sort(recs.begin(), recs.end(), [](const R& a, const R& b) {
      if (a.arr != b.arr) return a.arr < b.arr;
      if (a.addr != b.addr) return a.addr < b.addr;
      if (a.i != b.i) return a.i < b.i;
      return a.blk < b.blk;
    });
    std::vector<XbRec> loc;
    size_t s = 0;
    while (s < recs.size()) {
      size_t e = s;
      while (e < recs.size() && recs[e].arr == recs[s].arr && recs[e].addr == recs[s].addr) e++;
      loc.clear();
      for (size_t r = s; r < e; r++) loc.push_back({recs[r].i, recs[r].blk});
      cross_block_location(k, loc.data(), loc.size(), out);
      s = e;
    }
  }
}

// ----------------------------- conflicts, one array instance at a time
// The same relation, evaluated per (array, block) for the same-block
// relation and per (global array, address stripe) for the cross-block one,
// so that only one such part of the records is held at a time.  The parts
// are independent (a location lies in exactly one of them), so they are
// handed out to a pool of host threads, each with its own pair set; the sets
// are ORed at the end.  Stripe s of an array holds the addresses a with
// a % stripes == s; the stripe count keeps a part near g_part records.
int g_route = 0;              // 0: whole kernel at once; 1: one instance at a time
int g_threads = 0;            // threads of route 1 (0: every host core)
u64 g_part = 1ull << 25;      // records per cross-block part of route 1

void same_block_part(const or_kernel* k, u32 arr, u32 blk, std::vector<std::pair<u64, SbRec>>& recs,
                     PairSet& out) {
  recs.clear();
  for (u32 i = 0; i < k->n_points; i++) {
    if (k->points[i].kind != ACCESS || k->points[i].array != arr) continue;
    for (u32 t = 0; t < k->threads; t++)
      if (active(k, i, blk, t)) recs.push_back({address(k, i, blk, t), SbRec{i, t}});
  }
  std::sort(recs.begin(), recs.end(), [](const std::pair<u64, SbRec>& a,
                                         const std::pair<u64, SbRec>& b) {
    if (a.first != b.first) return a.first < b.first;
    if (a.second.i != b.second.i) return a.second.i < b.second.i;
    return a.second.t < b.second.t;
  });
  std::vector<SbRec> loc;
  size_t s = 0;
  while (s < recs.size()) {
    size_t e = s;
    while (e < recs.size() && recs[e].first == recs[s].first) e++;
    loc.clear();
    for (size_t r = s; r < e; r++) loc.push_back(recs[r].second);
    same_block_location(k, loc.data(), loc.size(), out);
    s = e;
  }
}

void cross_block_part(const or_kernel* k, u32 arr, u64 stripe, u64 stripes,
                      std::vector<std::pair<u64, XbRec>>& recs, PairSet& out) {
  recs.clear();
  for (u32 i = 0; i < k->n_points; i++) {
    if (k->points[i].kind != ACCESS || k->points[i].array != arr) continue;
    for (u32 blk = 0; blk < k->blocks; blk++)
      for (u32 t = 0; t < k->threads; t++)
        if (active(k, i, blk, t)) {
          const u64 a = address(k, i, blk, t);
          if (a % stripes == stripe) recs.push_back({a, XbRec{i, blk}});
        }
  }
  std::sort(recs.begin(), recs.end(), [](const std::pair<u64, XbRec>& a,
                                         const std::pair<u64, XbRec>& b) {
    if (a.first != b.first) return a.first < b.first;
    if (a.second.i != b.second.i) return a.second.i < b.second.i;
    return a.second.blk < b.second.blk;
  });
  std::vector<XbRec> loc;
  size_t s = 0;
  while (s < recs.size()) {
    size_t e = s;
    while (e < recs.size() && recs[e].first == recs[s].first) e++;
    loc.clear();
    for (size_t r = s; r < e; r++) loc.push_back(recs[r].second);
    cross_block_location(k, loc.data(), loc.size(), out);
    s = e;
  }
}

void conflicts_per_instance(const or_kernel* k, PairSet& out) {
  struct Task { u32 arr, blk; u64 stripe, stripes; bool cross; };
  std::vector<Task> tasks;
  for (u32 arr = 0; arr < k->n_arrays; arr++) {
    u64 n_cross = 0;
    bool used = false;
    for (u32 i = 0; i < k->n_points; i++) {
      if (k->points[i].kind != ACCESS || k->points[i].array != arr) continue;
      used = true;
      const u32 g = k->points[i].guard;
      u64 nt = 0, nb = 0;
      for (u32 t = 0; t < k->threads; t++)
        if (t % k->guards[g].m == k->guards[g].r) nt++;
      for (u32 blk = 0; blk < k->blocks; blk++)
        if (!k->block_guards || blk % k->block_guards[g].m == k->block_guards[g].r) nb++;
      n_cross += nt * nb;
    }
    if (!used) continue;
    for (u32 blk = 0; blk < k->blocks; blk++) tasks.push_back({arr, blk, 0, 1, false});
    if (k->arrays[arr].space == GLOBAL && k->blocks > 1) {
      const u64 stripes = std::max<u64>(1, (n_cross + g_part - 1) / g_part);
      for (u64 s = 0; s < stripes; s++) tasks.push_back({arr, 0, s, stripes, true});
    }
  }
  unsigned nth = g_threads > 0 ? (unsigned)g_threads : std::thread::hardware_concurrency();
  if (nth < 1) nth = 1;
  if (nth > tasks.size()) nth = (unsigned)std::max<size_t>(1, tasks.size());
  std::atomic<size_t> next(0);
  std::vector<PairSet> sets(nth, PairSet(k->n_points));
  auto work = [&](unsigned w) {
    std::vector<std::pair<u64, SbRec>> sb;
    std::vector<std::pair<u64, XbRec>> xb;
    for (;;) {
      const size_t q = next.fetch_add(1);
      if (q >= tasks.size()) break;
      const Task& t = tasks[q];
      if (t.cross) cross_block_part(k, t.arr, t.stripe, t.stripes, xb, sets[w]);
      else same_block_part(k, t.arr, t.blk, sb, sets[w]);
    }
  };
  std::vector<std::thread> pool;
  for (unsigned w = 1; w < nth; w++) pool.emplace_back(work, w);
  work(0);
  for (std::thread& th : pool) th.join();
  for (const PairSet& s : sets)
    for (size_t q = 0; q < s.bits.size(); q++) out.bits[q] |= s.bits[q];
}

// The conflict relation (independent of x) by the selected route.
void conflicts(const or_kernel* k, PairSet& out) {
  if (g_route == 1) conflicts_per_instance(k, out);
  else conflicts_grouped(k, out);
}

// Races under x from the conflict relation: the conflicting pairs no
// enabled barrier separates, in (level, i, j) order.
void races_from(const or_kernel* k, u64 x, const PairSet& conf, std::vector<or_pair>& out) {
  out.clear();
  for (int lv = 0; lv < 2; lv++)
    for (u32 i = 0; i < k->n_points; i++)
      for (u32 j = i; j < k->n_points; j++) {
        if (!conf.get(lv, i, j)) continue;
        if (separated(k, x, i, j, lv == 1)) continue;
        out.push_back({(uint16_t)i, (uint16_t)j, (uint8_t)lv, 0});
      }
}

// Races under x, emitted in (level, i, j) order.
void races(const or_kernel* k, u64 x, bool literal, std::vector<or_pair>& out) {
  PairSet ps(k->n_points);
  if (literal) {
    conflicts_literal(k, x, true, ps);
    out.clear();
    for (int lv = 0; lv < 2; lv++)
      for (u32 i = 0; i < k->n_points; i++)
        for (u32 j = i; j < k->n_points; j++)
          if (ps.get(lv, i, j)) out.push_back({(uint16_t)i, (uint16_t)j, (uint8_t)lv, 0});
    return;
  }
  conflicts(k, ps);
  races_from(k, x, ps, out);
}

// Positive clause of a race between i and j: the barrier variables of every
// occurrence strictly between them (only grid-level ones for a cross-block
// race).  An empty clause means no barrier can separate the pair.
u64 race_clause(const or_kernel* k, u32 i, u32 j, int lv) {
  u64 pos = 0;
  for (u32 u = i + 1; u < j; u++) {
    const or_point& p = k->points[u];
    if (p.kind != BARRIER) continue;
    if (lv == 1 && k->slots[p.slot].level != GRID) continue;
    pos |= 1ull << p.slot;
  }
  return pos;
}

bool clause_less(const or_clause& a, const or_clause& b) {
  return a.pos != b.pos ? a.pos < b.pos : a.neg < b.neg;
}

std::vector<or_clause> reduce(std::vector<or_clause> c) {
  std::sort(c.begin(), c.end(), clause_less);
  c.erase(std::unique(c.begin(), c.end(),
                      [](const or_clause& a, const or_clause& b) {
                        return a.pos == b.pos && a.neg == b.neg;
                      }),
          c.end());
  std::vector<or_clause> out;
  for (size_t a = 0; a < c.size(); a++) {
    bool subsumed = false;
    for (size_t b = 0; b < c.size() && !subsumed; b++) {
      if (a == b) continue;
      // c[b] subsumes c[a] when its literals are a subset of c[a]'s
      if ((c[b].pos & ~c[a].pos) == 0 && (c[b].neg & ~c[a].neg) == 0) subsumed = true;
    }
    if (!subsumed) out.push_back(c[a]);
  }
  return out;
}

// GenerateClause over every race under x, given the conflict relation.
std::vector<or_clause> clauses_from(const or_kernel* k, u64 x, const PairSet& conf) {
  std::vector<or_pair> rp;
  races_from(k, x, conf, rp);
  std::vector<or_clause> c;
  for (const or_pair& p : rp) c.push_back({race_clause(k, p.i, p.j, p.level), 0});
  u64 div = divergent_if_enabled(k, false) & x;
  for (u32 s = 0; s < 64; s++)
    if ((div >> s) & 1) c.push_back({0, 1ull << s});
  return reduce(c);
}

std::vector<or_clause> clauses_under(const or_kernel* k, u64 x) {
  PairSet conf(k->n_points);
  conflicts(k, conf);
  return clauses_from(k, x, conf);
}

// ------------------------------------------------------------------- solver
// key(x) = (W(x), popcount(x), x) lexicographic; as one integer it is the
// sum over enabled slots of w_s*2^71 + 2^64 + 2^s, which is additive.
u128 slot_key(const uint32_t* w, u32 s) {
  return ((u128)w[s] << 71) + ((u128)1 << 64) + ((u128)1 << s);
}

bool satisfies(const or_clause& c, u64 x) {
  return (x & c.pos) != 0 || (~x & c.neg) != 0;
}

int solve_exhaustive(const std::vector<or_clause>& c, const uint32_t* w, u32 S, u64* best_x) {
  bool found = false;
  u128 best = 0;
  for (u64 x = 0; x < (1ull << S); x++) {
    bool ok = true;
    for (const or_clause& cl : c)
      if (!satisfies(cl, x)) { ok = false; break; }
    if (!ok) continue;
    u128 key = 0;
    for (u32 s = 0; s < S; s++)
      if ((x >> s) & 1) key += slot_key(w, s);
    if (!found || key < best) { best = key; *best_x = x; found = true; }
  }
  return found ? OR_OK : OR_UNSAT;
}

struct BnB {
  const std::vector<or_clause>* c;
  const uint32_t* w;
  std::vector<u32> slots;  // component slots, ascending
  bool found = false;
  u128 best = 0;
  u64 best_x = 0;
  void dfs(size_t idx, u64 decided, u64 x, u128 key) {
    if (found && key >= best) return;  // every extension costs at least key
    for (const or_clause& cl : *c) {
      bool pos_dead = (cl.pos & ~(decided & ~x)) == 0;
      bool neg_dead = (cl.neg & ~(decided & x)) == 0;
      if (pos_dead && neg_dead) return;  // clause already falsified
    }
    if (idx == slots.size()) {
      found = true; best = key; best_x = x;
      return;
    }
    u64 bit = 1ull << slots[idx];
    dfs(idx + 1, decided | bit, x, key);
    dfs(idx + 1, decided | bit, x | bit, key + slot_key(w, slots[idx]));
  }
};

// Exact solve: slots in no positive literal stay false; the remaining
// clauses split into independent components (the key is additive), each
// solved by enumeration (<= 20 slots) or depth-first branch and bound.
int solve_reduced(const std::vector<or_clause>& in, const uint32_t* w, u32 S, u64* out) {
  u64 core = 0;
  for (const or_clause& c : in) core |= c.pos;
  std::vector<or_clause> cl;
  for (const or_clause& c : in) {
    if (c.neg & ~core) continue;  // satisfied: that slot stays false
    if ((c.pos | c.neg) == 0) return OR_UNSAT;
    cl.push_back(c);
  }
  // components by repeated closure over clause literal sets
  u64 left = core;
  u64 result = 0;
  while (left) {
    u64 comp = left & (~left + 1);
    bool grew = true;
    while (grew) {
      grew = false;
      for (const or_clause& c : cl) {
        u64 lit = c.pos | c.neg;
        if ((lit & comp) && (lit & ~comp)) { comp |= lit; grew = true; }
      }
    }
    left &= ~comp;
    std::vector<or_clause> cc;
    for (const or_clause& c : cl)
      if ((c.pos | c.neg) & comp) cc.push_back(c);
    std::vector<u32> ids;
    for (u32 s = 0; s < S; s++)
      if ((comp >> s) & 1) ids.push_back(s);
    if (ids.size() <= 20) {
      // enumerate the component's slots
      bool found = false;
      u128 best = 0;
      u64 best_x = 0;
      for (u64 m = 0; m < (1ull << ids.size()); m++) {
        u64 x = 0;
        u128 key = 0;
        for (size_t b = 0; b < ids.size(); b++)
          if ((m >> b) & 1) { x |= 1ull << ids[b]; key += slot_key(w, ids[b]); }
        bool ok = true;
        for (const or_clause& c : cc)
          if (!satisfies(c, x)) { ok = false; break; }
        if (ok && (!found || key < best)) { found = true; best = key; best_x = x; }
      }
      if (!found) return OR_UNSAT;
      result |= best_x;
    } else {
      BnB b;
      b.c = &cc; b.w = w; b.slots = ids;
      b.dfs(0, 0, 0, 0);
      if (!b.found) return OR_UNSAT;
      result |= b.best_x;
    }
  }
  *out = result;
  return OR_OK;
}

// Greedy minimal hitting set of the positive clauses (Section 2.4, the mhs
// strategy; the greedy of Johnson's set-cover approximation, weighted):
// repeatedly take the slot that hits the most clauses not yet hit per unit of
// weight (ties: lower slot id), then drop, in reverse order of choice, every
// chosen slot whose removal leaves all positive clauses hit.  Negative
// literals are ignored here.  An empty clause cannot be hit: OR_UNSAT.
int greedy_mhs(const std::vector<or_clause>& phi, const uint32_t* w, u32 S, u64* out) {
  std::vector<u64> pos;
  for (const or_clause& c : phi) {
    if (c.pos == 0 && c.neg == 0) return OR_UNSAT;
    if (c.pos && !c.neg) pos.push_back(c.pos);
  }
  std::vector<bool> hit(pos.size(), false);
  std::vector<u32> order;
  u64 x = 0;
  for (;;) {
    std::vector<u64> cnt(S, 0);
    bool open = false;
    for (size_t q = 0; q < pos.size(); q++) {
      if (hit[q]) continue;
      open = true;
      for (u32 s = 0; s < S; s++)
        if ((pos[q] >> s) & 1) cnt[s]++;
    }
    if (!open) break;
    int best = -1;
    for (u32 s = 0; s < S; s++) {
      if (cnt[s] == 0) continue;
      // cnt[s] / w[s] > cnt[best] / w[best], compared exactly
      if (best < 0 || cnt[s] * w[best] > cnt[best] * w[s]) best = (int)s;
    }
    if (best < 0) return OR_UNSAT;
    x |= 1ull << best;
    order.push_back((u32)best);
    for (size_t q = 0; q < pos.size(); q++)
      if ((pos[q] >> best) & 1) hit[q] = true;
  }
  for (size_t k = order.size(); k-- > 0;) {
    const u64 y = x & ~(1ull << order[k]);
    bool all = true;
    for (u64 c : pos)
      if (!(c & y)) { all = false; break; }
    if (all) x = y;
  }
  *out = x;
  return OR_OK;
}

u64 weight_of(const uint32_t* w, u32 S, u64 x) {
  u64 W = 0;
  for (u32 s = 0; s < S; s++)
    if ((x >> s) & 1) W += w[s];
  return W;
}

}  // namespace

// =========================================================== C entry points
extern "C" int or_validate(const or_kernel* k) { return validate(k); }

extern "C" int or_set_route(int route, int threads, uint64_t part_records) {
  const int old = g_route;
  if (route == 0 || route == 1) g_route = route;
  g_threads = threads > 0 ? threads : 0;
  g_part = part_records ? part_records : (1ull << 25);
  return old;
}

extern "C" int or_check(const or_kernel* k, uint64_t x, int literal, or_pair* pairs,
                        uint64_t cap, uint64_t* n_pairs, uint64_t* divergent,
                        uint64_t* n_records) {
  int v = validate(k);
  if (v != OR_OK) return v;
  std::vector<or_pair> rp;
  races(k, x, literal != 0, rp);
  if (n_records) *n_records = count_records(k);
  if (divergent) *divergent = divergent_if_enabled(k, literal != 0) & x;
  if (n_pairs) *n_pairs = rp.size();
  if (rp.size() > cap) return OR_ERR_CAPACITY;
  for (size_t n = 0; n < rp.size(); n++) pairs[n] = rp[n];
  return OR_OK;
}

extern "C" int or_pair_conflict(const or_kernel* k, uint32_t i, uint32_t j, int level) {
  if (validate(k) != OR_OK || i >= k->n_points || j >= k->n_points || i > j) return -1;
  const or_point& pa = k->points[i];
  const or_point& pb = k->points[j];
  if (pa.kind != ACCESS || pb.kind != ACCESS || pa.array != pb.array) return 0;
  if (!pa.is_write && !pb.is_write) return 0;
  if (level == 1 && !is_global(k, i)) return 0;
  // location -> distinct ids (thread for the same-block relation, block for
  // the cross-block one)
  struct E { u64 loc; u32 id; };
  auto collect = [&](u32 p, std::vector<E>& v) {
    for (u32 blk = 0; blk < k->blocks; blk++)
      for (u32 t = 0; t < k->threads; t++)
        if (active(k, p, blk, t)) {
          u64 a = address(k, p, blk, t);
          if (level == 0) v.push_back({((u64)blk << 32) | a, t});
          else v.push_back({a, blk});
        }
    std::sort(v.begin(), v.end(), [](const E& x, const E& y) {
      return x.loc != y.loc ? x.loc < y.loc : x.id < y.id;
    });
  };
  std::vector<E> A, B;
  collect(i, A);
  if (i == j) {
    for (size_t n = 1; n < A.size(); n++)
      if (A[n].loc == A[n - 1].loc && A[n].id != A[n - 1].id) return pa.is_write ? 1 : 0;
    return 0;
  }
  collect(j, B);
  size_t a = 0, b = 0;
  while (a < A.size() && b < B.size()) {
    if (A[a].loc < B[b].loc) { a++; continue; }
    if (B[b].loc < A[a].loc) { b++; continue; }
    u64 loc = A[a].loc;
    size_t ae = a, be = b;
    while (ae < A.size() && A[ae].loc == loc) ae++;
    while (be < B.size() && B[be].loc == loc) be++;
    bool a_one = A[a].id == A[ae - 1].id, b_one = B[b].id == B[be - 1].id;
    if (!(a_one && b_one && A[a].id == B[b].id)) return 1;
    a = ae; b = be;
  }
  return 0;
}

extern "C" int or_clauses(const or_kernel* k, uint64_t x, or_clause* out, uint64_t cap,
                          uint64_t* n) {
  int v = validate(k);
  if (v != OR_OK) return v;
  std::vector<or_clause> c = clauses_under(k, x);
  if (n) *n = c.size();
  if (c.size() > cap) return OR_ERR_CAPACITY;
  for (size_t q = 0; q < c.size(); q++) out[q] = c[q];
  return OR_OK;
}

extern "C" int or_full_clauses(const or_kernel* k, or_clause* out, uint64_t cap, uint64_t* n) {
  int v = validate(k);
  if (v != OR_OK) return v;
  // with no barrier enabled nothing separates, so the races under x = 0
  // are all conflicting pairs
  std::vector<or_clause> c;
  std::vector<or_pair> rp;
  races(k, 0, false, rp);
  for (const or_pair& p : rp) c.push_back({race_clause(k, p.i, p.j, p.level), 0});
  u64 div = divergent_if_enabled(k, false);
  for (u32 s = 0; s < 64; s++)
    if ((div >> s) & 1) c.push_back({0, 1ull << s});
  c = reduce(c);
  if (n) *n = c.size();
  if (c.size() > cap) return OR_ERR_CAPACITY;
  for (size_t q = 0; q < c.size(); q++) out[q] = c[q];
  return OR_OK;
}

extern "C" uint64_t or_reduce(or_clause* c, uint64_t n) {
  std::vector<or_clause> v(c, c + n);
  v = reduce(v);
  for (size_t q = 0; q < v.size(); q++) c[q] = v[q];
  return v.size();
}

extern "C" int or_min_barriers(const or_clause* c, uint64_t n, const uint32_t* weights,
                               uint32_t n_slots, int method, uint64_t* assign,
                               uint64_t* weight) {
  if (n_slots > 64 || (n && !c)) return OR_ERR_INVALID;
  for (u32 s = 0; s < n_slots; s++)
    if (weights[s] < 1) return OR_ERR_INVALID;
  u64 valid = n_slots == 64 ? ~0ull : ((1ull << n_slots) - 1);
  for (u64 q = 0; q < n; q++)
    if ((c[q].pos | c[q].neg) & ~valid) return OR_ERR_INVALID;
  std::vector<or_clause> cl(c, c + n);
  u64 x = 0;
  int st;
  if (method == 1) {
    if (n_slots > 26) return OR_ERR_INVALID;
    st = solve_exhaustive(cl, weights, n_slots, &x);
  } else {
    st = solve_reduced(cl, weights, n_slots, &x);
  }
  if (st == OR_OK) {
    if (assign) *assign = x;
    if (weight) *weight = weight_of(weights, n_slots, x);
  }
  return st;
}

// One Solve call of the repair loop: the exact optimum, or under the mhs
// strategy the greedy hitting set of the positive clauses, replaced by the
// exact optimum when it leaves a clause of phi unsatisfied (Section 2.4).
static int solve_step(const std::vector<or_clause>& phi, const uint32_t* w, u32 S, bool mhs,
                      u64* x) {
  if (!mhs) return solve_reduced(phi, w, S, x);
  int st = greedy_mhs(phi, w, S, x);
  if (st != OR_OK) return solve_reduced(phi, w, S, x);
  for (const or_clause& c : phi)
    if (!satisfies(c, *x)) return solve_reduced(phi, w, S, x);
  return OR_OK;
}

extern "C" int or_greedy_mhs(const or_clause* c, uint64_t n, const uint32_t* weights,
                             uint32_t n_slots, uint64_t* assign) {
  if (n_slots > 64 || (n && !c)) return OR_ERR_INVALID;
  std::vector<or_clause> cl(c, c + n);
  u64 x = 0;
  const int st = greedy_mhs(cl, weights, n_slots, &x);
  if (st == OR_OK && assign) *assign = x;
  return st;
}

extern "C" int or_repair(const or_kernel* k, const or_opts* o, or_result* out,
                         uint64_t* trajectory, uint32_t traj_cap) {
  int v = validate(k);
  if (v != OR_OK) return v;
  or_opts opt = o ? *o : or_opts{0, 1, 1, 0, 0};
  if (opt.solver > 1) return OR_ERR_INVALID;
  std::vector<uint32_t> w(k->n_slots);
  u64 pre = 0;
  for (u32 s = 0; s < k->n_slots; s++) {
    w[s] = k->slots[s].weight;
    if (k->slots[s].preexisting) pre |= 1ull << s;
  }
  // phi := true, plus the option units of Section 4.2 (Tab. 3): with
  // grid-level barriers disabled every grid slot is off; with inspection
  // disabled every pre-existing barrier is on (a pre-existing grid barrier
  // under both switches makes the first Solve UNSAT)
  std::vector<or_clause> phi;
  for (u32 s = 0; s < k->n_slots; s++) {
    if (!opt.grid && k->slots[s].level == GRID) phi.push_back({0, 1ull << s});
    if (!opt.inspect && k->slots[s].preexisting) phi.push_back({1ull << s, 0});
  }
  phi = reduce(phi);
  or_result r;
  std::memset(&r, 0, sizeof(r));
  u32 rounds = 0;
  bool mhs = opt.solver == 1;              // greedy rounds until the first SAFE
  u64 x = 0;
  // the conflict relation does not depend on the assignment: it is taken
  // once, and each Verify call keeps the pairs x leaves unseparated
  PairSet conf(k->n_points);
  conflicts(k, conf);
  int st = solve_step(phi, w.data(), k->n_slots, mhs, &x);   // Solve(phi)
  for (;;) {
    if (st == OR_UNSAT) { r.status = OR_UNSAT; break; }      // cannot be repaired
    if (opt.max_rounds && rounds == opt.max_rounds) { r.status = OR_ERR_ROUNDS; break; }
    if (trajectory && rounds < traj_cap) trajectory[rounds] = x;
    rounds++;
    std::vector<or_pair> rp;                                  // Verify(P_sol)
    races_from(k, x, conf, rp);
    u64 div = divergent_if_enabled(k, false) & x;
    if (rp.empty() && div == 0) {                             // SAFE
      if (mhs) {
        // the one exact query that makes the greedy result minimum; a
        // different optimum is verified in turn, with exact Solve from now on
        mhs = false;
        u64 xo = 0;
        solve_reduced(phi, w.data(), k->n_slots, &xo);
        if (xo != x) {
          x = xo;
          st = OR_OK;
          continue;
        }
      }
      r.status = OR_OK;
      r.assign = x;
      r.weight = weight_of(w.data(), k->n_slots, x);
      r.added = x & ~pre;
      r.removed = pre & ~x;
      break;
    }
    std::vector<or_clause> learned;                           // GenerateClause
    if (opt.policy == 0) {
      learned = clauses_from(k, x, conf);
    } else if (div) {
      learned.push_back({0, div & (~div + 1)});
    } else {
      learned.push_back({race_clause(k, rp[0].i, rp[0].j, rp[0].level), 0});
    }
    phi.insert(phi.end(), learned.begin(), learned.end());
    phi = reduce(phi);
    st = solve_step(phi, w.data(), k->n_slots, mhs, &x);
  }
  r.rounds = rounds;
  r.n_clauses = (u32)phi.size();
  if (out) *out = r;
  return r.status;
}

extern "C" int or_safe_literal(const or_kernel* k, uint64_t x) {
  if (validate(k) != OR_OK) return -1;
  PairSet ps(k->n_points);
  conflicts_literal(k, x, true, ps);
  for (size_t q = 0; q < ps.bits.size(); q++)
    if (ps.bits[q]) return 0;
  if (divergent_if_enabled(k, true) & x) return 0;
  return 1;
}

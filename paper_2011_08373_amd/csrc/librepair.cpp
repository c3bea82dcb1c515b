// librepair host side: descriptor validation and the per-kernel plan (field
// widths of the packed records, executing-thread counts, barrier tables).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <vector>

#include "common.h"
#include "launch.h"
#include "plan.h"

namespace rp {

static int g_digit_bits = 0;          // 0 = automatic
static int g_timing = 1;              // RP_TUNE_TIMING

int timing_level(int v, bool set) {
  const int old = g_timing;
  if (set) g_timing = v;
  return old;
}

static int g_digit_order = 1;         // RP_TUNE_DIGIT_ORDER

int digit_order(int v, bool set) {
  const int old = g_digit_order;
  if (set) g_digit_order = v;
  return old;
}

static int g_nodes_log2 = 28;         // RP_TUNE_SOLVER_NODES

int solver_nodes_log2(int v, bool set) {
  const int old = g_nodes_log2;
  if (set) g_nodes_log2 = v;
  return old;
}

int job_error_status(const JobState& st) {
  if (st.err == ERR_PHI_CAP || st.err == ERR_SCRATCH) return RP_ERR_CAPACITY;
  if (st.err == ERR_NODES) return RP_ERR_SEARCH;
  return RP_ERR_DEVICE;
}

int g_digit_bits_ref(int v, bool set) {
  const int old = g_digit_bits;
  if (set) g_digit_bits = v;
  return old;
}

static uint32_t bits_for(uint64_t maxval) {   // bits to hold 0..maxval
  return maxval == 0 ? 0u : (uint32_t)(64 - __builtin_clzll(maxval));
}

int validate_kernel(const rp_kernel* k) {
  if (!k) return RP_ERR_INVALID;
  if (k->blocks < 1 || k->threads < 1) return RP_ERR_INVALID;
  if (k->n_slots > 64 || k->n_points > (uint32_t)MAX_POINTS) return RP_ERR_INVALID;
  if ((k->n_arrays && !k->arrays) || (k->n_guards && !k->guards) ||
      (k->n_points && !k->points) || (k->n_slots && !k->slots))
    return RP_ERR_INVALID;
  uint64_t maxw = 1;
  for (uint32_t a = 0; a < k->n_arrays; a++) {
    if (k->arrays[a].words < 1 || k->arrays[a].space > 1) return RP_ERR_INVALID;
    maxw = std::max<uint64_t>(maxw, k->arrays[a].words);
  }
  bool bguard = false;
  for (uint32_t g = 0; g < k->n_guards; g++) {
    if (k->guards[g].m < 1 || k->guards[g].r >= k->guards[g].m) return RP_ERR_INVALID;
    if (k->block_guards) {
      if (k->block_guards[g].m < 1 || k->block_guards[g].r >= k->block_guards[g].m)
        return RP_ERR_INVALID;
      bguard |= k->block_guards[g].m > 1;
    }
  }
  for (uint32_t s = 0; s < k->n_slots; s++)
    if (k->slots[s].level > 1 || k->slots[s].preexisting > 1 || k->slots[s].weight < 1)
      return RP_ERR_INVALID;
  int32_t slot_guard[64];
  for (int s = 0; s < 64; s++) slot_guard[s] = -1;
  uint32_t next = 0;
  for (uint32_t i = 0; i < k->n_points; i++) {
    const rp_point& p = k->points[i];
    if (p.kind > RP_NOP) return RP_ERR_INVALID;
    if (p.kind == RP_ACCESS) {
      if (p.array >= k->n_arrays || p.guard >= k->n_guards || p.is_write > 1)
        return RP_ERR_INVALID;
    } else if (p.kind == RP_BARRIER) {
      if (p.slot >= k->n_slots || p.guard >= k->n_guards) return RP_ERR_INVALID;
      if (slot_guard[p.slot] < 0) {
        if (p.slot != next) return RP_ERR_INVALID;   // numbered by first occurrence
        next++;
        slot_guard[p.slot] = p.guard;
      } else if (slot_guard[p.slot] != (int32_t)p.guard) {
        return RP_ERR_INVALID;                         // one guard per slot
      }
    }
  }
  if (next != k->n_slots) return RP_ERR_INVALID;     // every slot occurs
  // (block conditions add one array id: the location of the padding records)
  const uint32_t total = bits_for(k->n_arrays ? k->n_arrays - 1 + bguard : 0) + bits_for(maxw - 1) +
                         bits_for(k->blocks - 1) + bits_for(k->n_points ? k->n_points - 1 : 0) +
                         bits_for(k->threads - 1);
  if (total > 64) return RP_ERR_INVALID;
  return RP_OK;
}

// Word compaction.  The sort only has to group records by location: the
// order of the locations themselves is free.  So each array's words are
// rotated (w -> (w + off) mod words) so that every word its accesses can
// touch lands in [0, span), and the word field of the records is only as
// wide as the largest span: fewer key bits, fewer or narrower radix passes.
// The touched words of a point lie in the arc of the circle of residues from
// the smallest to the largest value of a*t + b*k + c over its executing
// threads and blocks.  The circle is cut into CW_BINS bins; every bin an arc
// meets is marked, and the rotation moves the longest run of unmarked bins
// (words no access can touch) to the top of the range.  The rotation is
// folded into each point's c, so record generation is unchanged.
namespace {
constexpr uint32_t CW_BINS = 256;

// [min, max] of x * (r + m*u) over u in [0, n) (n >= 1); false on overflow
bool lin_range(int64_t x, uint64_t r, uint64_t m, uint64_t n, int64_t& lo, int64_t& hi) {
  int64_t a, b;
  if (r > (uint64_t)INT64_MAX || m * (n - 1) > (uint64_t)INT64_MAX) return false;
  if (__builtin_mul_overflow(x, (int64_t)r, &a)) return false;
  if (__builtin_mul_overflow(x, (int64_t)(m * (n - 1)), &b)) return false;
  int64_t l = 0, h = 0;
  if (__builtin_add_overflow(a, b < 0 ? b : 0, &l)) return false;
  if (__builtin_add_overflow(a, b > 0 ? b : 0, &h)) return false;
  lo = l;
  hi = h;
  return true;
}
}  // namespace

void compact_words(const rp_kernel* k, Plan& pl) {
  const uint32_t A = k->n_arrays;
  // per array: bins met by an arc (as a running-sum difference array), or
  // the whole circle
  static thread_local std::vector<int32_t> diff;
  static thread_local std::vector<uint8_t> full, used;
  diff.assign((size_t)A * (CW_BINS + 1), 0);
  full.assign(A, 0);
  used.assign(A, 0);
  // words per bin, as a shift when the array size is a power of two (the
  // usual case: no division per access)
  static thread_local std::vector<uint64_t> bws;
  static thread_local std::vector<int32_t> bsh;
  bws.resize(A);
  bsh.resize(A);
  for (uint32_t arr = 0; arr < A; arr++) {
    const uint64_t N = k->arrays[arr].words;
    bws[arr] = (N + CW_BINS - 1) / CW_BINS;
    const bool p2 = (N & (N - 1)) == 0 && (bws[arr] & (bws[arr] - 1)) == 0;
    bsh[arr] = p2 ? __builtin_ctzll(bws[arr]) : -1;
  }
  for (uint32_t i = 0; i < pl.P; i++) {
    const DPoint& d = pl.pts[i];
    if (d.kind != RP_ACCESS || d.cnt == 0) continue;
    const uint32_t arr = d.array;
    if (full[arr]) continue;
    const uint64_t N = k->arrays[arr].words;
    const uint64_t nblk = d.br < pl.B ? (pl.B - 1 - d.br) / d.bm + 1 : 0;
    if (nblk == 0) continue;
    used[arr] = 1;
    int64_t tlo, thi, blo, bhi, lo, hi;
    if (N > (1ull << 31) || !lin_range(d.a, d.r, d.m, d.cnt, tlo, thi) ||
        !lin_range(d.b, d.br, d.bm, nblk, blo, bhi) || __builtin_add_overflow(tlo, blo, &lo) ||
        __builtin_add_overflow(lo, (int64_t)d.c, &lo) || __builtin_add_overflow(thi, bhi, &hi) ||
        __builtin_add_overflow(hi, (int64_t)d.c, &hi) || (uint64_t)(hi - lo) + 1 >= N) {
      full[arr] = 1;   // rotated offsets must fit the int32 c; an arc round the circle
      continue;
    }
    const int32_t sh = bsh[arr];
    int64_t r;
    if (sh >= 0) {
      r = lo & (int64_t)(N - 1);
    } else {
      r = lo % (int64_t)N;
      if (r < 0) r += (int64_t)N;
    }
    const uint64_t bw = bws[arr];                       // words per bin
    const uint64_t s0 = (uint64_t)r, e0 = s0 + (uint64_t)(hi - lo);   // last word, may pass N
    int32_t* df = diff.data() + (size_t)arr * (CW_BINS + 1);
    auto mark = [&](uint64_t wa, uint64_t wb) {   // words [wa, wb] inside [0, N)
      df[sh >= 0 ? wa >> sh : wa / bw]++;
      df[(sh >= 0 ? wb >> sh : wb / bw) + 1]--;
    };
    if (e0 < N) {
      mark(s0, e0);
    } else {
      mark(s0, N - 1);
      mark(0, e0 - N);
    }
  }
  uint64_t span_max = 1;
  for (uint32_t arr = 0; arr < A; arr++) {
    const uint64_t N = k->arrays[arr].words;
    uint64_t off = 0, span = N;
    if (!used[arr] && !full[arr]) {
      span = 1;                                    // no access touches this array
    } else if (!full[arr]) {
      const uint64_t bw = bws[arr];
      const uint32_t nb = (uint32_t)((N + bw - 1) / bw);   // bins inside [0, N)
      const int32_t* df = diff.data() + (size_t)arr * (CW_BINS + 1);
      // longest circular run of unmarked bins: the runs inside [0, nb), and
      // the one that wraps (the unmarked tail joined to the unmarked head)
      static thread_local std::vector<uint8_t> marked;
      marked.resize(nb);
      int32_t run = 0;
      for (uint32_t j = 0; j < nb; j++) {
        run += df[j];
        marked[j] = run > 0;
      }
      uint32_t head = 0, tail = 0;
      while (head < nb && !marked[head]) head++;
      while (tail < nb && !marked[nb - 1 - tail]) tail++;
      uint32_t best_len = 0, best_end = 0, cur = 0;
      for (uint32_t j = 0; j < nb; j++) {
        if (!marked[j]) {
          if (++cur > best_len) {
            best_len = cur;
            best_end = j + 1 == nb ? 0 : j + 1;   // first bin after the run
          }
        } else {
          cur = 0;
        }
      }
      if (head < nb && head + tail > best_len) {   // the wrapping run
        best_len = head + tail;
        best_end = head;
      }
      if (head == nb) {
        span = 1;
      } else if (best_len > 0) {
        // words of the gap: bins best_end - best_len .. best_end - 1 (mod nb);
        // only the last bin of the circle can be narrower than bw
        const uint64_t last_w = N - (uint64_t)(nb - 1) * bw;
        const uint32_t first = best_end >= best_len ? best_end - best_len : best_end + nb - best_len;
        const bool has_last = first + best_len > nb || first + best_len == nb;
        const uint64_t gap = (uint64_t)(best_len - (has_last ? 1 : 0)) * bw + (has_last ? last_w : 0);
        const uint64_t next = (uint64_t)best_end * bw;    // first word after the gap
        off = (N - next % N) % N;
        span = N - gap;
      }
    }
    span_max = std::max(span_max, span);
    if (off == 0) continue;
    for (uint32_t i = 0; i < pl.P; i++) {
      DPoint& d = pl.pts[i];
      if (d.kind != RP_ACCESS || d.array != arr) continue;
      int64_t c = (int64_t)d.c % (int64_t)N;
      if (c < 0) c += (int64_t)N;
      d.c = (int32_t)(((uint64_t)c + off) % N);
    }
  }
  pl.nbits = bits_for(span_max - 1);
  pl.key_bits = pl.abits + pl.nbits;
}

void make_plan(const rp_kernel* k, Plan& pl) {
  pl.P = k->n_points;
  pl.S = k->n_slots;
  pl.B = k->blocks;
  pl.T = k->threads;
  uint64_t maxw = 1;
  for (uint32_t a = 0; a < k->n_arrays; a++) maxw = std::max<uint64_t>(maxw, k->arrays[a].words);
  bool bguard = false;
  if (k->block_guards)
    for (uint32_t g = 0; g < k->n_guards; g++) bguard |= k->block_guards[g].m > 1;
  // padding records of the same-block log (blocks that do not execute a
  // point) use array id n_arrays
  pl.pad_array = bguard ? k->n_arrays : 0;
  pl.abits = bits_for(k->n_arrays ? k->n_arrays - 1 + bguard : 0);
  pl.nbits = bits_for(maxw - 1);
  pl.bbits = bits_for(pl.B - 1);
  pl.pbits = bits_for(pl.P ? pl.P - 1 : 0);
  pl.tbits = bits_for(pl.T - 1);
  pl.key_shift = pl.tbits + pl.bbits + pl.pbits;
  pl.key_bits = pl.abits + pl.nbits;
  pl.pts.assign(pl.P, DPoint{});
  pl.wbits.assign((pl.P + 63) / 64, 0);
  pl.bits_any.assign(pl.P, 0);
  pl.bits_grid.assign(pl.P, 0);
  pl.cnt_pre.assign(pl.P + 1, 0);
  pl.gcnt_pre.assign(pl.P + 1, 0);
  pl.div_if_enabled = 0;
  pl.accesses = 0;
  for (uint32_t i = 0; i < pl.P; i++) {
    const rp_point& p = k->points[i];
    DPoint& d = pl.pts[i];
    d.kind = p.kind;
    d.flags = 0;
    d.cnt = 0;
    d.bm = 1;
    d.br = 0;
    uint64_t nblk = pl.B;           // blocks executing the point
    if (p.kind != RP_NOP) {
      const rp_guard& g = k->guards[p.guard];
      d.m = g.m;
      d.r = g.r;
      // threads t < T with t % m == r
      d.cnt = g.r < pl.T ? (pl.T - 1 - g.r) / g.m + 1 : 0;
      if (k->block_guards) {
        d.bm = k->block_guards[p.guard].m;
        d.br = k->block_guards[p.guard].r;
        nblk = d.br < pl.B ? (pl.B - 1 - d.br) / d.bm + 1 : 0;
      }
    }
    if (p.kind == RP_ACCESS) {
      const rp_array& a = k->arrays[p.array];
      d.a = p.a; d.b = p.b; d.c = p.c;
      d.words = a.words;
      d.array = p.array;
      if (p.is_write) {
        d.flags |= PF_WRITE;
        pl.wbits[i >> 6] |= 1ull << (i & 63);
      }
      if (a.space == RP_GLOBAL) d.flags |= PF_GLOBAL;
      if ((a.words & (a.words - 1)) == 0) d.flags |= PF_POW2;
      // a, b multiples of the array size (a mask test for power-of-two sizes)
      const int64_t nw = (int64_t)a.words;
      const bool p2 = (a.words & (a.words - 1)) == 0;
      if (p2 ? (((int64_t)p.a & (nw - 1)) == 0) : ((int64_t)p.a % nw == 0)) d.flags |= PF_TCONST;
      if (p2 ? (((int64_t)p.b & (nw - 1)) == 0) : ((int64_t)p.b % nw == 0)) d.flags |= PF_BCONST;
      pl.accesses += (uint64_t)d.cnt * nblk;
    }
    if (p.kind == RP_BARRIER) {
      pl.bits_any[i] = 1ull << p.slot;
      if (k->slots[p.slot].level == RP_GRID) pl.bits_grid[i] = 1ull << p.slot;
      // a block barrier must be reached by all threads of each block that
      // reaches it, a grid barrier by all threads of the grid
      const uint64_t reach = (uint64_t)d.cnt * nblk;
      const bool div = k->slots[p.slot].level == RP_GRID
                           ? reach > 0 && reach < (uint64_t)pl.B * pl.T
                           : nblk > 0 && d.cnt > 0 && d.cnt < pl.T;
      if (div) pl.div_if_enabled |= 1ull << p.slot;
    }
    // records emitted per point (the reductions are listed in common.h)
    uint64_t intra = 0, inter = 0;
    if (p.kind == RP_ACCESS) {
      const bool tc = d.flags & PF_TCONST;
      intra = tc ? std::min<uint64_t>(d.cnt, 2) : d.cnt;
      if ((d.flags & PF_GLOBAL) && pl.B > 1) {
        const uint64_t per_block = tc ? std::min<uint64_t>(d.cnt, 1) : d.cnt;
        const uint64_t blocks = (d.flags & PF_BCONST) ? std::min<uint64_t>(nblk, 2) : nblk;
        inter = per_block * blocks;
      }
    }
    pl.cnt_pre[i + 1] = pl.cnt_pre[i] + intra;
    pl.gcnt_pre[i + 1] = pl.gcnt_pre[i] + inter;
  }
  compact_words(k, pl);
  pl.weights.assign(pl.S, 0);
  pl.grid_slots = pl.pre_slots = 0;
  for (uint32_t s = 0; s < pl.S; s++) {
    pl.weights[s] = k->slots[s].weight;
    if (k->slots[s].level == RP_GRID) pl.grid_slots |= 1ull << s;
    if (k->slots[s].preexisting) pl.pre_slots |= 1ull << s;
  }
  pl.n_intra = pl.cnt_pre[pl.P] * pl.B;
  pl.n_inter = pl.gcnt_pre[pl.P];
}

// Automatic digit width: the fewest passes of at most 10 bits, each as
// narrow as that pass count allows (but at least 8 bits).
int pick_digit_bits(uint32_t key_bits) {
  if (g_digit_bits) return g_digit_bits;
  const uint32_t passes = std::max<uint32_t>(1, (key_bits + 9) / 10);
  const uint32_t rb = (key_bits + passes - 1) / passes;
  return (int)std::min<uint32_t>(10, std::max<uint32_t>(8, rb));
}

static int g_low_digit_bits = 6;      // RP_TUNE_LOW_DIGIT_BITS

int low_digit_bits(int v, bool set) {
  const int old = g_low_digit_bits;
  if (set) g_low_digit_bits = v;
  return old;
}

std::vector<DigitPass> digit_plan(uint32_t key_bits) {
  std::vector<DigitPass> v;     // lowest digit first
  if (key_bits == 0) return v;
  const uint32_t low = (uint32_t)g_low_digit_bits;
  // the rest of the key above a narrow lowest digit, in digits of at most
  // 10 bits but no fewer than 6 (the narrowest digit the kernels take)
  const uint32_t rest = key_bits > low ? key_bits - low : 0;
  const uint32_t n = (rest + 9) / 10;
  if (low != 0 && rest > 0 && rest >= 6 * n && g_digit_bits == 0) {
    v.push_back(DigitPass{0, low});
    uint32_t lo = low;
    for (uint32_t i = 0; i < n; i++) {
      const uint32_t w = rest / n + (i < rest % n ? 1u : 0u);
      v.push_back(DigitPass{lo, w});
      lo += w;
    }
  } else {
    const uint32_t rb = (uint32_t)pick_digit_bits(key_bits);
    for (uint32_t lo = 0; lo < key_bits; lo += rb) v.push_back(DigitPass{lo, rb});
  }
  if (g_digit_order != 0) std::reverse(v.begin(), v.end());
  return v;
}

}  // namespace rp

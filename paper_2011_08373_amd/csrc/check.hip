// Verify under an assignment x (the concrete counterpart of the verifier call
// of Alg. 1).
//
// ivl_kernel   one workgroup per job: interval ids = number of enabled
//              barrier occurrences before each point (any level, and grid
//              level only), the divergent enabled slots, and the first
//              partners under x resolved from the table j0 (or reset).
// conf_kernel  scan of the sorted logs under x for every racing pair (the
//              check call).  Records are in program order inside a location,
//              so the records of one interval are contiguous.  Two records
//              race when one writes and their ids (thread in the same-block
//              view, block in the cross-block view) differ.
//              conf_tiles_kernel lays the tiles over the logs of the jobs
//              still running.
// j0_kernel    the first partner of every point with no barrier enabled,
//              from which ivl_kernel resolves the first partners under any x.
// pairs_kernel turns the bitmap into the (level, i, j)-ordered pair list.
#include <algorithm>

#include "common.h"
#include "launch.h"

namespace rp {

constexpr int IVL_BLOCK = 1024;
constexpr int CONF_BLOCK = 256;
constexpr int CONF_WAVES = CONF_BLOCK / 64;
constexpr int CONF_CHUNKS = 16;                          // chunks of 64 records per wave and tile
constexpr uint32_t CONF_TILE = CONF_WAVES * CONF_CHUNKS * 64;   // records per tile

// mode IVL_RESOLVE: interval ids under x, then the first partners under x
//   from the assignment-independent table j0 (see below);
// mode IVL_CHECK: interval ids under x, first partners cleared, pair bitmap
//   cleared (the all-pairs scan follows);
// mode IVL_ZERO: interval ids of the empty assignment (one interval), first
//   partners cleared: the scan that follows fills j0.
//
// Why j0 suffices.  Inside one location the runs are in program order and
// interval ids never decrease along it, so the first run after r that
// conflicts with r in its whole location is either inside r's interval --
// then it is r's first partner under x -- or past its end, and then so is
// every conflicting run.  Taking the minimum over the runs of point i, the
// first partner of i under any x is j0[i] (its first partner when no barrier
// is enabled) if no enabled barrier lies strictly between i and j0[i], and
// none otherwise.
__global__ __launch_bounds__(IVL_BLOCK) void ivl_kernel(const Job* __restrict__ jobs, int mode) {
  __shared__ uint64_t wsum[IVL_BLOCK / 64];
  __shared__ uint32_t s_iv[2][MAX_POINTS];
  const Job& J = jobs[blockIdx.x];
  JobState* st = J.st;
  if (st->state != ST_RUN) return;
  const uint64_t x = mode == IVL_ZERO ? 0 : st->x;
  const uint32_t P = J.P;
  const int tid = threadIdx.x, lane = __lane_id(), w = tid >> 6;
  // four consecutive points per thread (P <= 4096)
  uint64_t cnt[4];
  uint64_t local = 0;
  for (int q = 0; q < 4; q++) {
    const uint32_t i = tid * 4 + q;
    uint64_t c = 0;
    if (i < P) {
      c = (J.bits_any[i] & x) ? 1 : 0;
      c |= (J.bits_grid[i] & x) ? (1ull << 32) : 0;
    }
    cnt[q] = c;
    local += c;
  }
  uint64_t inc = local;
  for (int off = 1; off < 64; off <<= 1) {
    uint64_t y = __shfl_up(inc, off);
    if (lane >= off) inc += y;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  uint64_t run = 0;
  for (int v = 0; v < w; v++) run += wsum[v];
  run += inc - local;
  for (int q = 0; q < 4; q++) {
    const uint32_t i = tid * 4 + q;
    if (i < P) {
      J.ivl[i] = s_iv[0][i] = (uint32_t)run;               // enabled occurrences before i
      J.ivl[P + i] = s_iv[1][i] = (uint32_t)(run >> 32);   // enabled GRID occurrences before i
    }
    run += cnt[q];
  }
  __syncthreads();
  if (mode == IVL_RESOLVE) {
    for (uint32_t r = tid; r < 2 * P; r += IVL_BLOCK) {
      const uint32_t lv = r >= P, i = r - lv * P;
      const uint32_t j = J.j0[r];
      J.minj[r] = (j < P && s_iv[lv][j] == s_iv[lv][i]) ? j : NONE32;
    }
  } else {
    for (uint32_t i = tid; i < 2 * P; i += IVL_BLOCK) J.minj[i] = NONE32;
  }
  if (mode == IVL_CHECK && J.bitmap) {
    const uint64_t nw = 2ull * P * J.wpr;
    for (uint64_t q = tid; q < nw; q += IVL_BLOCK) J.bitmap[q] = 0;
  }
  if (tid == 0 && mode != IVL_ZERO) st->divergent = x & J.div_if_enabled;
}

// j0 := the first partners just computed under the empty assignment.
__global__ __launch_bounds__(256) void save_j0_kernel(const Job* __restrict__ jobs) {
  const Job& J = jobs[blockIdx.x];
  for (uint32_t r = threadIdx.x; r < 2 * J.P; r += 256) J.j0[r] = J.minj[r];
}

__device__ __forceinline__ void set_pair(uint64_t* bm, uint32_t wpr, uint32_t P, uint32_t lv,
                                         uint32_t i, uint32_t j) {
  uint64_t* wp = bm + ((uint64_t)lv * P + i) * wpr + (j >> 6);
  const uint64_t bit = 1ull << (j & 63);
  if (!(*wp & bit)) atomicOr((unsigned long long*)wp, (unsigned long long)bit);
}

// Tile table of one scan: records of the logs of running jobs only, in
// segment order; one workgroup.
__global__ __launch_bounds__(1024) void conf_tiles_kernel(const Job* __restrict__ jobs,
                                                          ConfSeg* segs, uint32_t nseg,
                                                          uint32_t* total) {
  __shared__ uint32_t sm[16];
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  uint32_t run = 0;
  for (uint32_t b = 0; b < nseg; b += 1024) {
    const uint32_t q = b + threadIdx.x;
    uint32_t v = 0;
    if (q < nseg) {
      const ConfSeg& sg = segs[q];
      if (jobs[sg.job].st->state == ST_RUN) v = (uint32_t)((sg.n + CONF_TILE - 1) / CONF_TILE);
    }
    uint32_t inc = v;
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(inc, o);
      if (lane >= o) inc += y;
    }
    if (lane == 63) sm[w] = inc;
    __syncthreads();
    uint32_t pre = 0, all = 0;
    for (int k = 0; k < 16; k++) {
      if (k < w) pre += sm[k];
      all += sm[k];
    }
    if (q < nseg) segs[q].ctile_beg = run + pre + inc - v;
    run += all;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = run;
}

// A sorted log read as a sequence of one-record runs.  Record q becomes the
// entry  id | point << RUN_PT | writes << RUN_W | first-of-location << RUN_LOC
// (the id is the thread in the same-block view, the block in the cross-block
// view); two records of one point at one location are two runs of that point,
// which races with itself when it writes and their ids differ, and records
// equal in (point, id) never race with each other.  Past the end: the
// sentinel.
struct RecView {
  const uint64_t* log;
  uint64_t n;
  int psh, lsh, ish;       // point field, location, id shifts
  uint64_t imask;
  uint32_t pmask;
  const uint64_t* wb;      // write bit of each point (LDS)
};

__device__ __forceinline__ uint64_t shr(uint64_t v, int s) { return s >= 64 ? 0ull : v >> s; }

__device__ __forceinline__ RecView rec_view(const Job& J, const ConfSeg& sg, const uint64_t* wb) {
  RecView v;
  v.log = sg.log;
  v.n = sg.n;
  // same-block view: [array|word|block|point|thread]; location = (array, word, block)
  // cross-block view: [array|word|point|block|0];     location = (array, word)
  v.psh = sg.level == 0 ? (int)J.tbits : (int)(J.bbits + J.tbits);
  v.lsh = v.psh + (int)J.pbits;
  v.ish = sg.level == 0 ? 0 : (int)J.tbits;
  v.imask = sg.level == 0 ? ((1ull << J.tbits) - 1) : ((1ull << J.bbits) - 1);
  v.pmask = (1u << J.pbits) - 1u;
  v.wb = wb;
  return v;
}

__device__ __forceinline__ uint64_t make_entry(const RecView& v, uint64_t rec, uint64_t prev,
                                               uint64_t q) {
  if (q >= v.n) return RUN_SENTINEL;
  const uint32_t i = (uint32_t)shr(rec, v.psh) & v.pmask;
  const uint64_t id = shr(rec, v.ish) & v.imask;
  const uint64_t w = (v.wb[i >> 6] >> (i & 63)) & 1;
  const uint64_t loc = q == 0 || shr(rec, v.lsh) != shr(prev, v.lsh);
  return id | ((uint64_t)i << RUN_PT) | (w << RUN_W) | (loc << RUN_LOC);
}

__device__ __forceinline__ uint64_t entry_at(const RecView& v, uint64_t q) {
  if (q >= v.n) return RUN_SENTINEL;
  return make_entry(v, v.log[q], q > 0 ? v.log[q - 1] : 0, q);
}

// Stages records [b, b + 64*K) of a log as entries (all loads first).
template <int K>
__device__ __forceinline__ void stage_entries(const RecView& v, uint64_t b, uint64_t* buf) {
  const int lane = __lane_id();
  uint64_t r[K], p0;
#pragma unroll
  for (int k = 0; k < K; k++) {
    const uint64_t q = b + k * 64 + lane;
    r[k] = q < v.n ? v.log[q] : 0;
  }
  p0 = (lane == 0 && b > 0 && b - 1 < v.n) ? v.log[b - 1] : 0;
#pragma unroll
  for (int k = 0; k < K; k++) {
    uint64_t pr = __shfl_up(r[k], 1);
    const uint64_t last = k > 0 ? __shfl(r[k - 1], 63) : p0;   // every lane takes part
    if (lane == 0) pr = last;
    buf[k * 64 + lane] = make_entry(v, r[k], pr, b + k * 64 + lane);
  }
}

constexpr uint64_t NOPOS = ~0ull;

// First write run at or after position q, before the next location starts
// (NOPOS if none): wave-cooperative, 64 entries at a time; it ends at the
// end of the location.
__device__ uint64_t first_write_from(const RecView& v, uint64_t q) {
  const uint64_t n = v.n;
  for (; q < n; q += 64) {
    const uint64_t e = entry_at(v, q + __lane_id());
    const uint64_t wm = __ballot((e >> RUN_W) & 1);
    const uint64_t lm = __ballot((e >> RUN_LOC) & 1);
    if (wm && (!lm || __ffsll((unsigned long long)wm) < __ffsll((unsigned long long)lm)))
      return q + __ffsll((unsigned long long)wm) - 1;
    if (lm) return NOPOS;
  }
  return NOPOS;
}

// Racing pairs over a sorted log (the check call, which needs every pair).
// A sub-segment (one location, one interval) is a contiguous stretch of
// records.  Each wave stages a range of 1024 records in LDS (all loads in
// flight at once) and walks it in chunks of 64, one record per lane.  Inside
// a chunk, ballots give sub-segment starts and writes as 64-bit masks, so a
// lane takes the records after its own with mask operations; past its chunk
// it visits the rest of its sub-segment in order.
template <bool ALL>
__global__ __launch_bounds__(CONF_BLOCK) void conf_kernel(const Job* __restrict__ jobs,
                                                          const ConfSeg* __restrict__ segs,
                                                          int nseg,
                                                          const uint32_t* __restrict__ total_at) {
  __shared__ uint64_t s_buf[CONF_WAVES][CONF_CHUNKS * 64];
  __shared__ uint64_t s_wb[MAX_POINTS / 64];
  extern __shared__ uint32_t s_dyn[];        // [P] interval of each point, [P] first partner
  const uint32_t total = *total_at;
  const uint32_t per = (total + gridDim.x - 1) / gridDim.x;
  const uint32_t t0 = blockIdx.x * per;
  const uint32_t t1 = min(t0 + per, total);
  const int tid = threadIdx.x, lane = __lane_id(), wv = tid >> 6;
  const uint64_t gt = lane == 63 ? 0ull : (~0ull << (lane + 1));
  uint64_t* buf = s_buf[wv];
  int cur = -1;
  uint32_t* s_iv = s_dyn;
  uint32_t* s_minj = s_dyn;
  uint32_t P = 0;
  for (uint32_t tile = t0; tile < t1; tile++) {
    int lo = 0, hi = nseg - 1;   // largest segment with ctile_beg <= tile
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (segs[mid].ctile_beg <= tile) lo = mid; else hi = mid - 1;
    }
    if (lo != cur) {
      __syncthreads();
      if (!ALL && cur >= 0) {
        const Job& J = jobs[segs[cur].job];
        uint32_t* g = J.minj + (uint64_t)segs[cur].level * J.P;
        for (uint32_t i = tid; i < J.P; i += CONF_BLOCK)
          if (s_minj[i] != NONE32) atomicMin(&g[i], s_minj[i]);
      }
      __syncthreads();
      cur = lo;
      const Job& J = jobs[segs[cur].job];
      P = J.P;
      s_minj = s_dyn + P;
      const uint32_t* iv = J.ivl + (uint64_t)segs[cur].level * P;
      for (uint32_t i = tid; i < P; i += CONF_BLOCK) {
        s_iv[i] = iv[i];
        s_minj[i] = NONE32;
      }
      for (uint32_t q = tid; q < (P + 63) / 64; q += CONF_BLOCK) s_wb[q] = J.wbits[q];
      __syncthreads();
    }
    const ConfSeg& sg = segs[cur];
    const uint64_t n = sg.n;
    const uint64_t wbeg = (uint64_t)(tile - sg.ctile_beg) * CONF_TILE + (uint64_t)wv * (CONF_CHUNKS * 64);
    if (wbeg >= n) continue;
    const uint64_t wend = min(wbeg + (uint64_t)(CONF_CHUNKS * 64), n);
    const Job& J = jobs[sg.job];
    const uint32_t level = sg.level;
    const RecView V = rec_view(J, sg, s_wb);
    // stage the range
    stage_entries<CONF_CHUNKS>(V, wbeg, buf);
    // first write past the range in the same location
    uint64_t carry = first_write_from(V, wend);
    __builtin_amdgcn_wave_barrier();
    // entry at an absolute position: staged or global
    auto entry = [&](uint64_t q) -> uint64_t {
      return q < wend ? buf[q - wbeg] : entry_at(V, q);
    };
    const int nch = (int)((wend - wbeg + 63) / 64);
    for (int c = nch - 1; c >= 0; c--) {
      const uint64_t p0 = wbeg + (uint64_t)c * 64;
      const uint64_t e = buf[c * 64 + lane];
      const bool valid = !((e >> RUN_END) & 1);
      const uint32_t i = (uint32_t)(e >> RUN_PT) & 0xFFFu;
      const uint32_t iv = (valid && i < P) ? s_iv[i] : NONE32;
      const uint32_t prev = __shfl_up(iv, 1);
      const bool w = (e >> RUN_W) & 1, m = (e >> RUN_MULTI) & 1, ls = (e >> RUN_LOC) & 1;
      const uint64_t Bm = __ballot(ls || iv != prev);     // sub-segment starts (bit 0 unused)
      const uint64_t Lm = __ballot(ls);
      const uint64_t Wm = __ballot(w);
      const uint64_t Mm = __ballot(m);
      if (valid && i < P) {
        const uint32_t id = (uint32_t)e;
        uint32_t best = NONE32;
        if (w && m) {          // two threads (blocks) of one point on one word, one writes
          if (ALL) set_pair(J.bitmap, J.wpr, P, level, i, i);
          else best = i;
        }
        if (ALL || best == NONE32) {
          const uint64_t sC = Bm & gt;
          uint64_t cand = sC ? gt & ((sC & (~sC + 1)) - 1) : gt;
          if (!w) cand &= Wm;
          while (cand) {
            const int jj = __ffsll((unsigned long long)cand) - 1;
            cand &= cand - 1;
            const uint64_t ej = buf[c * 64 + jj];
            const uint32_t j = (uint32_t)(ej >> RUN_PT) & 0xFFFu;
            if (j < P && (m || ((Mm >> jj) & 1) || id != (uint32_t)ej)) {
              if (ALL) set_pair(J.bitmap, J.wpr, P, level, i, j);
              else { best = j; break; }
            }
          }
          // the sub-segment reaches the end of the chunk: look past it
          if (!sC && (ALL || best == NONE32)) {
            // first candidate past the chunk: the next run (a writing run,
            // or every run in "all" mode), else the carried first write
            uint64_t q = (w || ALL) ? p0 + 64 : carry;
            while (q < n) {
              const uint64_t ej = entry(q);
              if ((ej >> RUN_LOC) & 1) break;
              const uint32_t j = (uint32_t)(ej >> RUN_PT) & 0xFFFu;
              if (j >= P || s_iv[j] != iv) break;        // next interval
              const bool wj = (ej >> RUN_W) & 1;
              if ((w || wj) && (m || ((ej >> RUN_MULTI) & 1) || id != (uint32_t)ej)) {
                if (ALL) set_pair(J.bitmap, J.wpr, P, level, i, j);
                else { best = j; break; }
              }
              q++;
            }
          }
        }
        if (!ALL && best != NONE32 && s_minj[i] > best) atomicMin(&s_minj[i], best);
      }
      // carry for the chunk before: first write from p0 on, before a location start
      if (Wm && (!Lm || __ffsll((unsigned long long)Wm) < __ffsll((unsigned long long)Lm)))
        carry = p0 + __ffsll((unsigned long long)Wm) - 1;
      else if (Lm)
        carry = NOPOS;
    }
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  if (!ALL && cur >= 0) {
    const Job& J = jobs[segs[cur].job];
    uint32_t* g = J.minj + (uint64_t)segs[cur].level * J.P;
    for (uint32_t i = tid; i < J.P; i += CONF_BLOCK)
      if (s_minj[i] != NONE32) atomicMin(&g[i], s_minj[i]);
  }
}

// ---------------------------------------------------------------------------
// First partners with no barrier enabled (the table j0), in one pass over the
// sorted logs with no per-record walk.
//
// With every barrier off a location is one sub-segment, and the first
// partner of record r is the first later record q of its location with
// (W_r or W_q) and id_r != id_q.  Call a "streak" a maximal stretch of records
// of one id (a new location or a new id starts one) and, among the writes of
// a location, a "write streak" likewise.  Then the first partner of
//   - a write is the next record, or if that has the same id, the end of its
//     streak;
//   - a read is the first write f after it, or if f has the same id, the end
//     of f's write streak.
// (A point racing with itself needs no case of its own: its next record with
// another id is that partner.)  Each wave stages 1024 records in LDS and walks
// them in chunks of 64 from the last to the first; inside a chunk the
// candidates come from ballot masks, past it from four wave-wide carries (the
// next record, its streak end, the first write ahead and that write's
// write-streak end), set up at the end of the range by short probes that
// stop at the end of the location.
__device__ __forceinline__ uint64_t bits_above(int k) {   // bits k+1..63
  return k >= 63 ? 0ull : (~0ull << (k + 1));
}
__device__ __forceinline__ uint64_t bits_below(int k) {   // bits 0..k-1
  return k <= 0 ? 0ull : (k >= 64 ? ~0ull : ((1ull << k) - 1));
}
__device__ __forceinline__ int low_bit(uint64_t m) { return __ffsll((unsigned long long)m) - 1; }

__device__ __forceinline__ bool run_single_same(uint64_t a, uint64_t b) {   // same single id
  return !((a >> RUN_MULTI) & 1) && !((b >> RUN_MULTI) & 1) && (uint32_t)a == (uint32_t)b;
}

// First position q > a with a streak start (relative to q-1), or n.
__device__ uint64_t probe_streak_end(const RecView& v, uint64_t a) {
  const uint64_t n = v.n;
  for (uint64_t base = a + 1; base < n; base += 64) {
    const uint64_t q = base + __lane_id();
    const uint64_t e = entry_at(v, q);
    const uint64_t pr = entry_at(v, q - 1);
    const bool x = q < n && (((e >> RUN_LOC) & 1) || !run_single_same(e, pr));
    const uint64_t xm = __ballot(x);
    if (xm) return base + low_bit(xm);
  }
  return n;
}

// First write q > f with (M_q or id_q != id_f) before the location ends, or NOPOS.
__device__ uint64_t probe_write_streak_end(const RecView& v, uint64_t f, uint64_t ef) {
  const uint64_t n = v.n;
  for (uint64_t base = f + 1; base < n; base += 64) {
    const uint64_t e = entry_at(v, base + __lane_id());
    const uint64_t hm = __ballot(((e >> RUN_W) & 1) && !run_single_same(e, ef) &&
                                 !((e >> RUN_END) & 1));
    const uint64_t lm = __ballot((e >> RUN_LOC) & 1);
    if (hm && (!lm || low_bit(hm) < low_bit(lm))) return base + low_bit(hm);
    if (lm) return NOPOS;
  }
  return NOPOS;
}

__global__ __launch_bounds__(CONF_BLOCK) void j0_kernel(const Job* __restrict__ jobs,
                                                        const ConfSeg* __restrict__ segs, int nseg,
                                                        const uint32_t* __restrict__ total_at) {
  __shared__ uint64_t s_buf[CONF_WAVES][CONF_CHUNKS * 64];
  __shared__ uint64_t s_wb[MAX_POINTS / 64];
  extern __shared__ uint32_t s_dyn[];        // [P] first partner
  const uint32_t total = *total_at;
  const uint32_t per = (total + gridDim.x - 1) / gridDim.x;
  const uint32_t t0 = blockIdx.x * per;
  const uint32_t t1 = min(t0 + per, total);
  const int tid = threadIdx.x, lane = __lane_id(), wv = tid >> 6;
  // lane masks: lanes below, above, above lane + 1, at or below
  const uint64_t lt = bits_below(lane), gt = bits_above(lane), gt1 = bits_above(lane + 1);
  const uint64_t le = bits_below(lane + 1);
  uint64_t* buf = s_buf[wv];
  int cur = -1;
  uint32_t* s_minj = s_dyn;
  uint32_t P = 0;
  for (uint32_t tile = t0; tile < t1; tile++) {
    int lo = 0, hi = nseg - 1;   // largest segment with ctile_beg <= tile
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (segs[mid].ctile_beg <= tile) lo = mid; else hi = mid - 1;
    }
    if (lo != cur) {
      __syncthreads();
      if (cur >= 0) {
        const Job& J = jobs[segs[cur].job];
        uint32_t* g = J.minj + (uint64_t)segs[cur].level * J.P;
        for (uint32_t i = tid; i < J.P; i += CONF_BLOCK)
          if (s_minj[i] != NONE32) atomicMin(&g[i], s_minj[i]);
      }
      __syncthreads();
      cur = lo;
      const Job& J = jobs[segs[cur].job];
      P = J.P;
      for (uint32_t i = tid; i < P; i += CONF_BLOCK) s_minj[i] = NONE32;
      for (uint32_t q = tid; q < (P + 63) / 64; q += CONF_BLOCK) s_wb[q] = J.wbits[q];
      __syncthreads();
    }
    const ConfSeg& sg = segs[cur];
    const uint64_t n = sg.n;
    const uint64_t wbeg = (uint64_t)(tile - sg.ctile_beg) * CONF_TILE + (uint64_t)wv * (CONF_CHUNKS * 64);
    if (wbeg >= n) continue;
    const uint64_t wend = min(wbeg + (uint64_t)(CONF_CHUNKS * 64), n);
    const RecView V = rec_view(jobs[sg.job], sg, s_wb);
    stage_entries<CONF_CHUNKS>(V, wbeg, buf);
    __builtin_amdgcn_wave_barrier();
    auto entry = [&](uint64_t q) -> uint64_t {
      return (q >= wbeg && q < wend) ? buf[q - wbeg] : entry_at(V, q);
    };
    auto accepts = [&](uint64_t ea, uint64_t eb) -> bool {   // different threads (blocks)
      return !run_single_same(ea, eb);
    };
    // carries for the positions from the end of the range on
    uint64_t A = wend;                                   // next run
    const uint64_t eA0 = entry_at(V, wend);
    bool XA = wend >= n || ((eA0 >> RUN_LOC) & 1) || (uint32_t)eA0 != (uint32_t)buf[wend - 1 - wbeg];
    uint64_t SEA = wend < n ? probe_streak_end(V, wend) : n;   // its streak end
    uint64_t FW = first_write_from(V, wend);             // first write ahead
    uint64_t NWS = FW != NOPOS ? probe_write_streak_end(V, FW, entry_at(V, FW)) : NOPOS;
    const int nch = (int)((wend - wbeg + 63) / 64);
    const uint64_t first_pred = wbeg > 0 ? entry_at(V, wbeg - 1) : RUN_SENTINEL;
    for (int c = nch - 1; c >= 0; c--) {
      const uint64_t p0 = wbeg + (uint64_t)c * 64;
      const uint64_t e = buf[c * 64 + lane];
      const bool valid = !((e >> RUN_END) & 1);
      const uint32_t i = (uint32_t)(e >> RUN_PT) & 0xFFFu;
      const bool w = (e >> RUN_W) & 1, ls = (e >> RUN_LOC) & 1;
      // predecessor (lane 0: the last record of the chunk before, or before the range)
      uint64_t pe = __shfl_up(e, 1);
      if (lane == 0) pe = c > 0 ? buf[c * 64 - 1] : first_pred;
      const bool x = ls || (uint32_t)e != (uint32_t)pe;
      const uint64_t Xm = __ballot(x);
      const uint64_t Lm = __ballot(ls);
      const uint64_t Wm = __ballot(w && valid);
      // write-streak starts among the writes of the chunk (relative to the
      // previous write of the chunk; only queried after an earlier write)
      const uint64_t pwm = Wm & lt;
      const int pw = pwm ? 63 - __clzll((long long)pwm) : 0;
      const uint64_t epw = __shfl(e, pw);
      const bool xw = w && valid && pwm &&
                      ((Lm & bits_above(pw) & le) || (uint32_t)e != (uint32_t)epw);
      const uint64_t XWm = __ballot(xw);
      if (valid && i < P) {
        // first candidate: the next record (a write) or the first write
        // after this record (a read); second, when the first has the same
        // id: the end of that record's streak (a write) or write streak
        // (a read)
        const uint64_t hw = Wm & gt, hl = Lm & gt;
        bool f_in = false;
        uint64_t c1;
        if (w) {
          c1 = p0 + lane + 1;
        } else if (hw && (!hl || low_bit(hw) < low_bit(hl))) {
          c1 = p0 + low_bit(hw);
          f_in = true;
        } else {
          c1 = hl ? NOPOS : FW;
        }
        uint32_t best = NONE32;
        if (c1 < n) {
          const uint64_t e1 = entry(c1);
          if (!((e1 >> RUN_LOC) & 1)) {
            if ((uint32_t)e1 != (uint32_t)e) {
              best = (uint32_t)(e1 >> RUN_PT) & 0xFFFu;
            } else {
              uint64_t c2;
              if (w) {
                const uint64_t hx = Xm & gt1;     // streak starts after lane + 1
                c2 = hx ? p0 + low_bit(hx) : (lane < 63 && XA ? A : SEA);
              } else if (f_in) {
                const int fl = (int)(c1 - p0);
                const uint64_t hxw = XWm & bits_above(fl), hl2 = Lm & bits_above(fl);
                if (hxw && (!hl2 || low_bit(hxw) < low_bit(hl2))) c2 = p0 + low_bit(hxw);
                else if (hl2) c2 = NOPOS;
                else c2 = (FW != NOPOS && (uint32_t)entry(FW) != (uint32_t)e1) ? FW : NWS;
              } else {
                c2 = NWS;
              }
              if (c2 < n) {
                const uint64_t e2 = entry(c2);
                if (!((e2 >> RUN_LOC) & 1)) best = (uint32_t)(e2 >> RUN_PT) & 0xFFFu;
              }
            }
          }
        }
        if (best < P && s_minj[i] > best) atomicMin(&s_minj[i], best);
      }
      // carries for the positions from p0 on
      const uint64_t hx0 = Xm & ~1ull;
      const uint64_t nSEA = hx0 ? p0 + low_bit(hx0) : (XA ? A : SEA);
      const bool nXA = Xm & 1ull;
      const int fl0 = Lm ? low_bit(Lm) : 64;
      const uint64_t wb = Wm & bits_below(fl0);
      if (wb) {
        const int f0 = low_bit(wb);
        const uint64_t ef0 = buf[c * 64 + f0];
        const uint64_t hxw = XWm & bits_above(f0), hl2 = Lm & bits_above(f0);
        uint64_t nn;
        if (hxw && (!hl2 || low_bit(hxw) < low_bit(hl2))) nn = p0 + low_bit(hxw);
        else if (hl2) nn = NOPOS;
        else nn = (FW != NOPOS && accepts(ef0, entry(FW))) ? FW : NWS;
        FW = p0 + f0;
        NWS = nn;
      } else if (Lm) {
        FW = NOPOS;
        NWS = NOPOS;
      }
      A = p0;
      XA = nXA;
      SEA = nSEA;
    }
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  if (cur >= 0) {
    const Job& J = jobs[segs[cur].job];
    uint32_t* g = J.minj + (uint64_t)segs[cur].level * J.P;
    for (uint32_t i = tid; i < J.P; i += CONF_BLOCK)
      if (s_minj[i] != NONE32) atomicMin(&g[i], s_minj[i]);
  }
}

// Bitmap rows (level, i) in order -> pair list; one workgroup, rows in
// contiguous chunks per thread so the block scan keeps row order.
__global__ __launch_bounds__(1024) void pairs_kernel(const Job* __restrict__ jobs, rp_pair* out,
                                                     uint64_t* total) {
  __shared__ uint64_t wsum[16];
  const Job& J = jobs[0];
  const uint32_t rows = 2 * J.P;
  const uint32_t per = (rows + 1023) / 1024;
  const int tid = threadIdx.x, lane = __lane_id(), w = tid >> 6;
  uint64_t local = 0;
  for (uint32_t q = 0; q < per; q++) {
    const uint32_t row = tid * per + q;
    if (row >= rows) break;
    const uint64_t* rw = J.bitmap + (uint64_t)row * J.wpr;
    for (uint32_t c = 0; c < J.wpr; c++) local += __popcll(rw[c]);
  }
  uint64_t inc = local;
  for (int off = 1; off < 64; off <<= 1) {
    uint64_t y = __shfl_up(inc, off);
    if (lane >= off) inc += y;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  uint64_t pos = 0, tot = 0;
  for (int v = 0; v < 16; v++) {
    if (v < w) pos += wsum[v];
    tot += wsum[v];
  }
  pos += inc - local;
  if (tid == 0) *total = tot;
  for (uint32_t q = 0; q < per; q++) {
    const uint32_t row = tid * per + q;
    if (row >= rows) break;
    const uint32_t lv = row / J.P, i = row % J.P;
    const uint64_t* rw = J.bitmap + (uint64_t)row * J.wpr;
    for (uint32_t c = 0; c < J.wpr; c++) {
      uint64_t m = rw[c];
      while (m) {
        const uint32_t b = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        rp_pair pr;
        pr.i = (uint16_t)i;
        pr.j = (uint16_t)(c * 64 + b);
        pr.level = (uint8_t)lv;
        pr.pad = 0;
        out[pos++] = pr;
      }
    }
  }
}

uint32_t conf_tile_size() { return CONF_TILE; }

hipError_t launch_ivl(const Job* jobs, uint32_t njobs, int mode, hipStream_t s) {
  if (njobs == 0) return hipSuccess;
  ivl_kernel<<<njobs, IVL_BLOCK, 0, s>>>(jobs, mode);
  return hipGetLastError();
}

hipError_t launch_save_j0(const Job* jobs, uint32_t njobs, hipStream_t s) {
  if (njobs == 0) return hipSuccess;
  save_j0_kernel<<<njobs, 256, 0, s>>>(jobs);
  return hipGetLastError();
}

hipError_t launch_conf_tiles(const Job* jobs, ConfSeg* segs, int nseg, uint32_t* tiles,
                             hipStream_t s) {
  if (nseg == 0) return hipSuccess;
  conf_tiles_kernel<<<1, 1024, 0, s>>>(jobs, segs, (uint32_t)nseg, tiles);
  return hipGetLastError();
}

hipError_t launch_conf(const Job* jobs, const ConfSeg* segs, int nseg, uint32_t max_points,
                       const uint32_t* tiles, hipStream_t s) {
  if (nseg == 0) return hipSuccess;
  const size_t dyn = 2 * (size_t)(max_points ? max_points : 1) * sizeof(uint32_t);
  int dev = 0, ncu = 256, per_cu = 0;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, conf_kernel<true>, CONF_BLOCK, dyn) !=
          hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  const uint32_t grid = (uint32_t)ncu * (uint32_t)std::min(per_cu, 8);
  conf_kernel<true><<<grid, CONF_BLOCK, dyn, s>>>(jobs, segs, nseg, tiles);
  return hipGetLastError();
}

hipError_t launch_j0(const Job* jobs, const ConfSeg* segs, int nseg, uint32_t max_points,
                     const uint32_t* tiles, hipStream_t s) {
  if (nseg == 0) return hipSuccess;
  const size_t dyn = (size_t)(max_points ? max_points : 1) * sizeof(uint32_t);
  int dev = 0, ncu = 256, per_cu = 0;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, j0_kernel, CONF_BLOCK, dyn) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  const uint32_t grid = (uint32_t)ncu * (uint32_t)std::min(per_cu, 8);
  j0_kernel<<<grid, CONF_BLOCK, dyn, s>>>(jobs, segs, nseg, tiles);
  return hipGetLastError();
}

hipError_t launch_pairs(const Job* job, rp_pair* out, uint64_t* total, hipStream_t s) {
  pairs_kernel<<<1, 1024, 0, s>>>(job, out, total);
  return hipGetLastError();
}

}  // namespace rp

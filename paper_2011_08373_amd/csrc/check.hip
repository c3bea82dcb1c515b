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
  gptr<uint64_t> log;
  uint64_t n;
  int psh, ish;            // point and id field shifts (< 64)
  uint32_t pmask, imask;   // point and id field masks
  uint64_t locm, idm;      // location bits, id bits of a record
  const uint16_t* pw;      // per point: the point | its write bit << 12 (LDS)
};

__device__ __forceinline__ uint64_t shr(uint64_t v, int s) { return s >= 64 ? 0ull : v >> s; }

__device__ __forceinline__ RecView rec_view(const Job& J, const ConfSeg& sg, const uint16_t* pw) {
  RecView v;
  v.log = as_global(sg.log);
  v.n = sg.n;
  // same-block view: [array|word|block|point|thread]; location = (array, word, block)
  // cross-block view: [array|word|point|block|0];     location = (array, word)
  const int psh = sg.level == 0 ? (int)J.tbits : (int)(J.bbits + J.tbits);
  const int lsh = psh + (int)J.pbits;
  const int ish = sg.level == 0 ? 0 : (int)J.tbits;
  const uint64_t imask = sg.level == 0 ? ((1ull << J.tbits) - 1) : ((1ull << J.bbits) - 1);
  // a field at bit 64 or above is empty
  v.psh = psh < 64 ? psh : 0;
  v.pmask = psh < 64 ? (1u << J.pbits) - 1u : 0u;
  v.ish = ish < 64 ? ish : 0;
  v.imask = ish < 64 ? (uint32_t)imask : 0u;
  v.locm = lsh < 64 ? ~0ull << lsh : 0ull;
  v.idm = ish < 64 ? imask << ish : 0ull;
  v.pw = pw;
  return v;
}

// Entry of a record from the record itself and the one before it in the log
// (first: it starts the log).
__device__ __forceinline__ uint64_t make_entry_of(const RecView& v, uint64_t rec, uint64_t prev,
                                                  bool first) {
  const uint64_t df = rec ^ prev;
  const uint32_t i = (uint32_t)(rec >> v.psh) & v.pmask;
  const uint32_t id = (uint32_t)(rec >> v.ish) & v.imask;
  const uint32_t loc = first || (df & v.locm) != 0;
  const uint32_t x = loc | ((df & v.idm) != 0);
  const uint32_t hi = v.pw[i] | (x << (RUN_X - 32)) | (loc << (RUN_LOC - 32));
  return (uint64_t)id | ((uint64_t)hi << 32);
}

__device__ __forceinline__ uint64_t make_entry(const RecView& v, uint64_t rec, uint64_t prev,
                                               uint64_t q) {
  if (q >= v.n) return RUN_SENTINEL;
  return make_entry_of(v, rec, prev, q == 0);
}

__device__ __forceinline__ uint64_t entry_at(const RecView& v, uint64_t q) {
  if (q >= v.n) return RUN_SENTINEL;
  return make_entry(v, v.log[q], q > 0 ? v.log[q - 1] : 0, q);
}

// Stages records [b, b + 64*K) of a log as entries (all loads first); lane 0
// returns the raw record before b (0 when b == 0).
template <int K>
__device__ __forceinline__ uint64_t stage_entries(const RecView& v, uint64_t b, uint64_t* buf,
                                                  uint64_t* ent = nullptr) {
  const int lane = __lane_id();
  uint64_t r[K];
  const uint64_t p0 = (lane == 0 && b > 0 && b - 1 < v.n) ? v.log[b - 1] : 0;
  if (b + 64 * K <= v.n) {        // the whole span inside the log: no per-record test
#pragma unroll
    for (int k = 0; k < K; k++) r[k] = v.log[b + k * 64 + lane];
#pragma unroll
    for (int k = 0; k < K; k++) {
      uint64_t pr = __shfl_up(r[k], 1);
      const uint64_t last = k > 0 ? __shfl(r[k - 1], 63) : p0;   // every lane takes part
      if (lane == 0) pr = last;
      const uint64_t en = make_entry_of(v, r[k], pr, k == 0 && lane == 0 && b == 0);
      buf[k * 64 + lane] = en;
      if (ent) ent[k] = en;
    }
  } else {
#pragma unroll
    for (int k = 0; k < K; k++) {
      const uint64_t q = b + k * 64 + lane;
      r[k] = q < v.n ? v.log[q] : 0;
    }
#pragma unroll
    for (int k = 0; k < K; k++) {
      uint64_t pr = __shfl_up(r[k], 1);
      const uint64_t last = k > 0 ? __shfl(r[k - 1], 63) : p0;   // every lane takes part
      if (lane == 0) pr = last;
      const uint64_t en = make_entry(v, r[k], pr, b + k * 64 + lane);
      buf[k * 64 + lane] = en;
      if (ent) ent[k] = en;
    }
  }
  return p0;
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
  __shared__ uint16_t s_pw[MAX_POINTS];      // point | write bit << 12, per point
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
      for (uint32_t q = tid; q < P; q += CONF_BLOCK)
        s_pw[q] = (uint16_t)(q | (((J.wbits[q >> 6] >> (q & 63)) & 1) << (RUN_W - 32)));
      __syncthreads();
    }
    const ConfSeg& sg = segs[cur];
    const uint64_t n = sg.n;
    const uint64_t wbeg = (uint64_t)(tile - sg.ctile_beg) * CONF_TILE + (uint64_t)wv * (CONF_CHUNKS * 64);
    if (wbeg >= n) continue;
    const uint64_t wend = min(wbeg + (uint64_t)(CONF_CHUNKS * 64), n);
    const Job& J = jobs[sg.job];
    const uint32_t level = sg.level;
    const RecView V = rec_view(J, sg, s_pw);
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
      const bool w = (e >> RUN_W) & 1, ls = (e >> RUN_LOC) & 1;
      const uint64_t Bm = __ballot(ls || iv != prev);     // sub-segment starts (bit 0 unused)
      const uint64_t Lm = __ballot(ls);
      const uint64_t Wm = __ballot(w);
      if (valid && i < P) {
        const uint32_t id = (uint32_t)e;
        uint32_t best = NONE32;
        {
          const uint64_t sC = Bm & gt;
          uint64_t cand = sC ? gt & ((sC & (~sC + 1)) - 1) : gt;
          if (!w) cand &= Wm;
          while (cand) {
            const int jj = __ffsll((unsigned long long)cand) - 1;
            cand &= cand - 1;
            const uint64_t ej = buf[c * 64 + jj];
            const uint32_t j = (uint32_t)(ej >> RUN_PT) & 0xFFFu;
            if (j < P && id != (uint32_t)ej) {
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
              if ((w || wj) && id != (uint32_t)ej) {
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
//   - a write is the end of its streak: the first later record with another
//     id (the records before it share the write's id);
//   - a read is the first write f after it, or if f has the same id, the end
//     of f's write streak.
// (A point racing with itself needs no case of its own: its next record with
// another id is that partner.)
//
// Each wave takes a contiguous part of a log and walks it backward in chunks
// of 64 records, one record per lane, straight from registers: a ballot of
// each compare gives the location starts, streak starts and writes of the
// chunk as 64-bit masks; a lane's first candidate is the lowest set bit above
// it, whose point and id come from that lane by a cross-lane permute; past the
// chunk, wave-wide carries (scalar registers) hold what lies ahead: the
// partner point of the first streak start, and the first write with its id
// and the end of its write streak.  The carries at the end of a part come
// from a short forward walk over the records after it, which stops at the end
// of the location it starts in.

__device__ __forceinline__ uint32_t low_bit64(uint64_t m) {   // 64 if m == 0
  return m ? (uint32_t)__builtin_ctzll(m) : 64u;
}
__device__ __forceinline__ uint64_t above(uint32_t k) {       // bits k+1..63 (none for k >= 63)
  return k >= 63 ? 0ull : (~0ull << (k + 1));
}
// Lowest set bit of a wave-uniform mask, 0xffffffff when it is empty (the
// scalar find-first-one gives exactly that, with no test of its own).
__device__ __forceinline__ uint32_t first_one(uint64_t m) {
  uint32_t r;
  asm("s_ff1_i32_b64 %0, %1" : "=s"(r) : "s"(m));
  return r;
}
__device__ __forceinline__ uint64_t ballot64(bool p) { return __builtin_amdgcn_ballot_w64(p); }
// This lane's bit of the wave mask m (the mask itself serves as the lane
// condition of a select, with no per-lane test).
__device__ __forceinline__ bool lane_in(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }
// A wave-uniform value held in a vector register, so that an instruction can
// take it beside a scalar operand (an instruction reads one scalar register).
__device__ __forceinline__ uint32_t in_vgpr(uint32_t v) {
  uint32_t r;
  asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "s"(v));
  return r;
}
// Lanes below the lowest set lane of m (all lanes when m is empty).
__device__ __forceinline__ uint64_t below_first(uint64_t m) { return (m & (0ull - m)) - 1ull; }


// The record one lane down (lane 0 gets `first`, the record before the chunk).
__device__ __forceinline__ uint64_t lane_before(uint64_t v, uint64_t first) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  // DPP wave shift right by one lane; the lane with no source keeps `old`
  lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)first, (int)lo, 0x138, 0xF, 0xF, false);
  hi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(first >> 32), (int)hi, 0x138, 0xF,
                                             0xF, false);
  return ((uint64_t)hi << 32) | lo;
}

// The record one lane down, where lane 0 gets lane 63 of `last` (the chunk
// before): a wave rotate of `last` puts its lane 63 into lane 0, and the wave
// shift of v leaves that lane as it is.
__device__ __forceinline__ uint64_t lane_before_chunk(uint64_t v, uint64_t last) {
  const int rl = __builtin_amdgcn_mov_dpp((int)(uint32_t)last, 0x13C, 0xF, 0xF, false);
  const int rh = __builtin_amdgcn_mov_dpp((int)(uint32_t)(last >> 32), 0x13C, 0xF, 0xF, false);
  const uint32_t lo =
      (uint32_t)__builtin_amdgcn_update_dpp(rl, (int)(uint32_t)v, 0x138, 0xF, 0xF, false);
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_update_dpp(rh, (int)(uint32_t)(v >> 32), 0x138, 0xF, 0xF, false);
  return ((uint64_t)hi << 32) | lo;
}

// Value of v in lane l mod 64 (ds_bpermute takes the source lane from the
// byte address divided by four, modulo the wave size).
__device__ __forceinline__ uint32_t from_lane(uint32_t v, uint32_t l) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute((int)(l << 2), (int)v);
}

// Fields of the records of one log.  With LO32 (the point and id fields lie
// in the low 32 bits of every record of the launch) a field is one bit-field
// extract of the low word, and the id test one 32-bit compare.
struct J0Fields {
  int psh, ish;            // point and id field shifts (< 64)
  uint32_t pmask, imask;   // point and id field masks
  uint32_t pw, iw;         // point and id field widths
  uint64_t locm, idm;      // location bits, id bits of a record
  uint64_t lmax;           // a record pair differs in its location iff their xor > lmax
};

__device__ __forceinline__ J0Fields j0_fields(const Job& J, const ConfSeg& sg) {
  // same-block view: [array|word|block|point|thread]; location = (array, word, block)
  // cross-block view: [array|word|point|block|0];     location = (array, word)
  J0Fields f;
  const int psh = sg.level == 0 ? (int)J.tbits : (int)(J.bbits + J.tbits);
  const int lsh = psh + (int)J.pbits;
  const int ish = sg.level == 0 ? 0 : (int)J.tbits;
  const uint64_t imask = sg.level == 0 ? ((1ull << J.tbits) - 1) : ((1ull << J.bbits) - 1);
  f.psh = psh < 64 ? psh : 0;
  f.pmask = psh < 64 ? (1u << J.pbits) - 1u : 0u;
  f.ish = ish < 64 ? ish : 0;
  f.imask = ish < 64 ? (uint32_t)imask : 0u;
  f.pw = psh < 64 ? J.pbits : 0u;
  f.iw = ish < 64 ? (sg.level == 0 ? J.tbits : J.bbits) : 0u;
  f.locm = lsh < 64 ? ~0ull << lsh : 0ull;
  f.idm = ish < 64 ? imask << ish : 0ull;
  f.lmax = lsh < 64 ? (1ull << lsh) - 1ull : ~0ull;
  return f;
}

// One chunk of 64 records (lane l: record base + l) decoded into wave masks
// and per-lane fields.  valid: this lane holds a record (all lanes but those
// past the log end; always with FULL).  Lanes past the end read as location
// starts, so every search stops there, and as non-writes in Wm (their own W,
// point and id are never used).  Lane 0 of a chunk that starts the log needs
// no flag of its own: a location start there only bounds searches from lanes
// before it, and there are none.
struct J0Chunk {
  uint64_t Lm, Xm, Wm;     // location starts, streak starts (Lm included), writes
  uint32_t pt, id;
  bool W, L, valid;        // this lane: a write, a location start, a record
};

template <bool FULL, bool LO32>
__device__ __forceinline__ J0Chunk j0_decode(const J0Fields& f, const uint8_t* s_w, uint64_t rec,
                                             uint64_t prev, bool valid) {
  J0Chunk c;
  const uint64_t df = rec ^ prev;
  bool idc;
  if constexpr (LO32) {
    c.pt = __builtin_amdgcn_ubfe((uint32_t)rec, (uint32_t)f.psh, f.pw);
    c.id = __builtin_amdgcn_ubfe((uint32_t)rec, (uint32_t)f.ish, f.iw);
    idc = ((uint32_t)df & (uint32_t)f.idm) != 0;
  } else {
    c.pt = (uint32_t)(rec >> f.psh) & f.pmask;
    c.id = (uint32_t)(rec >> f.ish) & f.imask;
    idc = (df & f.idm) != 0;
  }
  c.W = s_w[c.pt] != 0;
  c.valid = FULL || valid;
  c.L = df > f.lmax || !c.valid;
  c.Lm = ballot64(c.L);
  c.Xm = c.Lm | ballot64(idc);
  c.Wm = ballot64(c.W && c.valid);
  return c;
}

// What lies ahead of a position, for the records before it in its location.
struct J0Carry {
  uint32_t x;              // partner point of the first streak start (NONE32: a location start)
  uint32_t fw, fw_id;      // first write before the location ends (NONE32: none), its id
  uint32_t ws;             // end of that write's write streak: the first later write with
                           // another id before the location ends (NONE32: none)
};

// The carries at the start of a chunk from the chunk and the carries at its
// end, as scalar selects with no branch: every lane index below is taken mod
// 64, so the reads of an empty mask's "first" lane are harmless and their
// results are not selected.
__device__ __forceinline__ void j0_carry_update(J0Carry& cr, const J0Chunk& c) {
  // the first streak start: its partner point, none at a location start
  const uint32_t x0 = first_one(c.Xm) & 63u;
  const uint32_t px = __builtin_amdgcn_readlane(c.pt, x0);
  const uint32_t x = c.Xm == 0 ? cr.x : (((c.Lm >> x0) & 1) ? NONE32 : px);
  // the first write or location start
  const uint64_t wl = c.Wm | c.Lm;
  const uint32_t b = first_one(wl) & 63u;
  const uint32_t fid = __builtin_amdgcn_readlane(c.id, b);
  const uint32_t fpt = __builtin_amdgcn_readlane(c.pt, b);
  const uint64_t after = ~1ull << b;                         // lanes above b
  // (a ballot of a plain compare is the compare's own mask)
  const uint64_t hm = ballot64(c.id != fid) & c.Wm & after;
  const uint64_t lm = c.Lm & after;
  // the write's write-streak end: the first later write with another id
  // before the location ends, else none if the location ends in the chunk,
  // else what lies past the chunk
  const uint32_t h = first_one(hm), l = first_one(lm);       // 0xffffffff: none
  const uint32_t ph = __builtin_amdgcn_readlane(c.pt, h & 63u);
  // (with no write ahead, fw and ws are both NONE32, so either is right)
  const uint32_t past = cr.fw_id != fid ? cr.fw : cr.ws;
  const uint32_t nws = h < l ? ph : (l != NONE32 ? NONE32 : past);
  const bool loc = (c.Lm >> b) & 1;                          // a location start first
  cr.x = x;
  if (wl != 0) {
    cr.fw = loc ? NONE32 : fpt;
    cr.fw_id = loc ? cr.fw_id : fid;
    cr.ws = loc ? NONE32 : nws;
  }
}

// Carries at position s (a multiple of 64 from the log start, or n) from
// the records at and after it: a forward walk, chunk by chunk, until the
// first streak start, the first write or location start and that write's
// write-streak end are known.  It stops at the end of the location it
// starts in (or of the log).
template <bool LO32>
__device__ J0Carry j0_carry_at(gptr<uint64_t> log, uint64_t n, uint64_t s,
                               const J0Fields& f, const uint8_t* s_w) {
  J0Carry cr{NONE32, NONE32, 0, NONE32};
  if (s >= n) return cr;
  const uint32_t lane = __lane_id();
  bool have_x = false, have_fw = false, have_ws = false;
  uint64_t prev_last = log[s - 1];          // s > 0: a part never starts the walk at 0
  for (uint64_t base = s; base < n + 64 && !(have_x && have_ws); base += 64) {
    const uint64_t q = base + lane;
    const uint64_t rec = q < n ? log[q] : 0;
    const uint64_t prev = lane_before(rec, prev_last);
    prev_last = __shfl(rec, 63);
    const J0Chunk c = j0_decode<false, LO32>(f, s_w, rec, prev, q < n);
    if (!have_x && c.Xm) {
      const uint32_t x0 = low_bit64(c.Xm);
      cr.x = ((c.Lm >> x0) & 1) ? NONE32 : __builtin_amdgcn_readlane(c.pt, x0);
      have_x = true;
    }
    uint64_t from = ~0ull;                  // lanes after the first write, if it is here
    if (!have_fw) {
      const uint64_t wl = c.Wm | c.Lm;
      if (!wl) continue;
      const uint32_t b = low_bit64(wl);
      have_fw = true;
      if ((c.Lm >> b) & 1) {
        have_ws = true;                     // a location start first: no write ahead
        continue;
      }
      cr.fw = __builtin_amdgcn_readlane(c.pt, b);
      cr.fw_id = __builtin_amdgcn_readlane(c.id, b);
      from = above(b);
    }
    if (!have_ws) {
      const uint64_t hm = ballot64(c.W && c.id != cr.fw_id) & c.Wm & from;
      const uint64_t lm = c.Lm & from;
      if (hm && low_bit64(hm) < low_bit64(lm)) {
        cr.ws = __builtin_amdgcn_readlane(c.pt, low_bit64(hm));
        have_ws = true;
      } else if (lm) {
        have_ws = true;                     // ws stays NONE32
      }
    }
  }
  return cr;
}

// Chunks per range: the records of a range are all loaded before any is
// decoded (that many loads in flight per lane).  With PIPE the next range's
// loads are issued before the current range is scanned.
constexpr int J0_CHUNKS = 8;

// One range of chunks, scanned backward: first partners into s_minj, carries
// moved to the range start.  rev[j]: this lane's record of chunk
// J0_CHUNKS - 1 - j (the order of the scan, which is also the order of the
// loads: the compiler issues the loads of an array in index order); before:
// the record before the range (any value at the log start).  FULL: the
// range has all J0_CHUNKS chunks, every one inside the log (no per-chunk or
// per-lane end test).
template <bool FULL, bool LO32>
__device__ __forceinline__ void j0_range(const J0Fields& F, const uint8_t* s_w, uint32_t* s_minj,
                                         uint32_t P, const uint64_t (&rev)[J0_CHUNKS],
                                         uint64_t before, uint64_t wbeg, int nch, uint64_t n,
                                         J0Carry& cr) {
  const uint32_t lane = __lane_id();
  const uint64_t gt = above(lane);                                  // lanes above
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));   // lanes below
#pragma unroll
  for (int k = J0_CHUNKS - 1; k >= 0; k--) {
    if (!FULL && k >= nch) continue;
    const uint64_t base = wbeg + (uint64_t)k * 64;
    const uint64_t rk = rev[J0_CHUNKS - 1 - k];
    const uint64_t prev = k > 0 ? lane_before_chunk(rk, rev[J0_CHUNKS - k])   // chunk k - 1
                                : lane_before(rk, before);
    const J0Chunk c = j0_decode<FULL, LO32>(F, s_w, rk, prev, FULL || base + lane < n);
    // first candidate: for a write the first streak start after it, for
    // a read the first write or location start after it; in the chunk it is
    // read from its lane as a partner value (the point, or none where a
    // location starts), past the chunk it is the carried one.  The lane's
    // mask, Xm for a write and WL = Wm | Lm for a read, taken above the lane,
    // is a bit-field insert of Xm into WL & gt under gt of the writes (one
    // scalar operand per instruction).  Which lanes find a candidate in the
    // chunk (those below the highest bit of their mask) and the rest of the
    // lane logic are wave masks, so that each per-lane select takes its
    // mask from scalar registers.
    const uint64_t WL = c.Wm | c.Lm;
    const uint32_t gwl = c.W ? (uint32_t)gt : 0u, gwh = c.W ? (uint32_t)(gt >> 32) : 0u;
    const uint32_t tlo = (uint32_t)WL & (uint32_t)gt, thi = (uint32_t)(WL >> 32) & (uint32_t)(gt >> 32);
    const uint32_t mlo = (gwl & (uint32_t)c.Xm) | (~gwl & tlo);
    const uint32_t mhi = (gwh & (uint32_t)(c.Xm >> 32)) | (~gwh & thi);
    const uint32_t c1 = low_bit64(((uint64_t)mhi << 32) | mlo);
    const bool in1 = c1 < 64;
    const uint64_t in1m = ballot64(in1);
    const uint32_t pv = lane_in(c.Lm) ? NONE32 : c.pt;
    const uint32_t pv1 = from_lane(pv, c1), id1 = from_lane(c.id, c1);
    const uint32_t cfw = cr.fw, cfw_id = cr.fw_id, cws = cr.ws;
    const uint32_t past = c.W ? cr.x : cfw;                         // x for a write, fw for a read
    const uint32_t cand = in1 ? pv1 : past;
    // a read whose first write has its own id: the partner is the end of
    // that write's write streak (carried when the write lies past the chunk)
    const uint64_t eqm = (in1m & ballot64(id1 == c.id)) | (~in1m & ballot64(cfw_id == c.id));
    const uint64_t secm = ~c.Wm & ballot64(cand != NONE32) & eqm;
    const bool second = lane_in(secm);
    uint32_t best = second ? cws : cand;
    // Reads whose first write f lies in the chunk with the read's own id:
    // the partner is the first write after f with another id before the
    // location ends.  With write-streak starts (writes whose id differs from
    // that of the write before them in the chunk; a location start in
    // between is met first) it is the first such start or location start
    // after f, else it lies past the chunk: the carried first write if its
    // id differs, else the end of that write's write streak.  Only chunks
    // where some read needs it take this step.
    const uint64_t need = secm & in1m & (FULL ? ~0ull : ballot64(c.valid));
    if (need) {
      // the nearest write below this lane (any lane where there is none:
      // those lanes are not above the chunk's first write, and WSm drops them)
      const uint64_t pm = c.Wm & lt;
      const uint32_t pw = 63u - (uint32_t)__builtin_clzg(pm, 64);
      const uint32_t idpw = from_lane(c.id, pw);
      // (the chunk has a write here: some read's first write lies in it)
      const uint64_t WSm = ballot64(idpw != c.id) & c.Wm & (~1ull << (first_one(c.Wm) & 63u));
      // lanes above c1 (c1 < 64 where needed; bit 63 shifts out at c1 = 63)
      const uint32_t k2 = low_bit64((WSm | c.Lm) & (~1ull << c1));
      const uint32_t pv2 = from_lane(pv, k2);
      if (lane_in(need))
        best = k2 < 64 ? pv2 : (cfw_id != id1 ? cfw : cws);   // (no write ahead: both NONE32)
    }
    // every lane takes part (NONE32 leaves the minimum as it is), so the
    // add needs no lane mask
    atomicMin(&s_minj[c.pt], FULL || c.valid ? best : NONE32);
    j0_carry_update(cr, c);
  }
}

template <bool PIPE, bool LO32>
__global__ __launch_bounds__(CONF_BLOCK) void j0_kernel(const Job* __restrict__ jobs,
                                                        const ConfSeg* __restrict__ segs, int nseg,
                                                        const uint32_t* __restrict__ total_at) {
  // the write bit of each point (bytes; a static array, so that its LDS
  // address is known when compiling and a point is read with no address
  // arithmetic) and the first partner of each point (u32, [P] dynamic)
  __shared__ uint8_t s_w[MAX_POINTS];
  extern __shared__ uint32_t s_dyn[];
  // the tiles' 64-record chunks, split evenly over the workgroups (whole
  // tiles per workgroup would leave some with none when there are few tiles
  // per workgroup)
  constexpr uint32_t TC = CONF_TILE / 64;     // chunks per tile
  const uint64_t nunits = (uint64_t)*total_at * TC;
  const uint64_t u0 = nunits * blockIdx.x / gridDim.x;
  const uint64_t u1 = nunits * (blockIdx.x + 1) / gridDim.x;
  // the wave index is uniform across the wave: say so, so that the range
  // bounds and the chunk loop stay scalar
  const int tid = threadIdx.x, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t lane = __lane_id();
  int cur = -1;
  uint32_t* s_minj = s_dyn;
  uint32_t P = 0;
  for (uint64_t u = u0; u < u1;) {
    const uint32_t tile = (uint32_t)(u / TC);
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
      for (uint32_t i = tid; i < P; i += CONF_BLOCK) {
        s_minj[i] = NONE32;
        s_w[i] = (uint8_t)((J.wbits[i >> 6] >> (i & 63)) & 1);
      }
      __syncthreads();
    }
    const ConfSeg& sg = segs[cur];
    const uint64_t n = sg.n;
    const gptr<uint64_t> log = as_global(sg.log);
    J0Fields F = j0_fields(jobs[sg.job], sg);
    if constexpr (LO32) {
      F.pw = in_vgpr(F.pw);
      F.iw = in_vgpr(F.iw);
    }
    // this workgroup's chunks of the segment, as one record span cut into
    // one contiguous part per wave (whole chunks)
    const uint64_t ub = (uint64_t)sg.ctile_beg * TC;
    const uint64_t uend = cur + 1 < nseg ? min(u1, (uint64_t)segs[cur + 1].ctile_beg * TC) : u1;
    const uint64_t rbeg = min((u - ub) * 64, n);
    const uint64_t rend = min((uend - ub) * 64, n);
    u = uend;
    const uint64_t part = (rend - rbeg + CONF_WAVES * 64 - 1) / (CONF_WAVES * 64) * 64;
    const uint64_t s0 = min(rbeg + (uint64_t)wv * part, rend);
    const uint64_t s1 = min(s0 + part, rend);
    if (s0 >= s1) continue;
    J0Carry cr = j0_carry_at<LO32>(log, n, s1, F, s_w);
    // the part backward in ranges of J0_CHUNKS chunks
    const int nr = (int)((s1 - s0 + J0_CHUNKS * 64 - 1) / (J0_CHUNKS * 64));
    // a range's loads: the record before it (needed last) first, then its
    // chunks in the order they are scanned (the last first), so the scan can
    // start before the whole range has arrived; none is conditional (chunks
    // past the part are read but not scanned, lanes past the log end read
    // its last record, and neither value is used)
    auto load_range = [&](int r, uint64_t (&dst)[J0_CHUNKS], uint64_t& bef) {
      const uint64_t wb = s0 + (uint64_t)r * (J0_CHUNKS * 64);
      bef = log[wb > 0 ? wb - 1 : 0];
      if (wb + J0_CHUNKS * 64 <= n) {
        // wholly inside the log: one address, the chunks at immediate offsets
        const gptr<uint64_t> p = log + wb + lane;
#pragma unroll
        for (int j = 0; j < J0_CHUNKS; j++) dst[j] = p[(J0_CHUNKS - 1 - j) * 64];
      } else {
#pragma unroll
        for (int j = 0; j < J0_CHUNKS; j++) {
          const uint64_t q = wb + (uint64_t)(J0_CHUNKS - 1 - j) * 64 + lane;
          dst[j] = log[q < n ? q : n - 1];
        }
      }
    };
    auto scan_range = [&](const uint64_t (&rv)[J0_CHUNKS], uint64_t before, uint64_t wbeg,
                          int nch) {
      if (nch == J0_CHUNKS && wbeg + (uint64_t)nch * 64 <= n)
        j0_range<true, LO32>(F, s_w, s_minj, P, rv, before, wbeg, nch, n, cr);
      else
        j0_range<false, LO32>(F, s_w, s_minj, P, rv, before, wbeg, nch, n, cr);
    };
    uint64_t rev[J0_CHUNKS], before;
    load_range(nr - 1, rev, before);
    for (int r = nr - 1; r >= 0; r--) {
      const uint64_t wbeg = s0 + (uint64_t)r * (J0_CHUNKS * 64);
      // (a 32-bit scalar count, so that each chunk's test is one scalar compare)
      const int nch = __builtin_amdgcn_readfirstlane(
          (int)min((uint64_t)J0_CHUNKS, (s1 - wbeg + 63) / 64));
      if constexpr (PIPE) {
        uint64_t nxt[J0_CHUNKS], nbef = 0;
        if (r > 0) load_range(r - 1, nxt, nbef);
        scan_range(rev, before, wbeg, nch);
        if (r > 0) {
#pragma unroll
          for (int j = 0; j < J0_CHUNKS; j++) rev[j] = nxt[j];
          before = nbef;
        }
      } else {
        scan_range(rev, before, wbeg, nch);
        if (r > 0) load_range(r - 1, rev, before);
      }
    }
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

static int g_j0_variant = 1;   // 0: loads of a range after the range before it is scanned,
                               // 1: the next range's loads in flight during the scan
int j0_variant(int v, bool set) {
  const int old = g_j0_variant;
  if (set) g_j0_variant = v;
  return old;
}

static int g_j0_fields = 0;    // 0: 32-bit fields where they fit, 1: always 64-bit records
int j0_fields_variant(int v, bool set) {
  const int old = g_j0_fields;
  if (set) g_j0_fields = v;
  return old;
}

template <bool PIPE, bool LO32>
static hipError_t j0_go(const Job* jobs, const ConfSeg* segs, int nseg, uint32_t max_points,
                        const uint32_t* tiles, hipStream_t s) {
  // [P] first partners (u32); the write bits are a static array
  const size_t dyn = (size_t)(max_points ? max_points : 1) * sizeof(uint32_t);
  int dev = 0, ncu = 256, per_cu = 0;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, j0_kernel<PIPE, LO32>, CONF_BLOCK, dyn) !=
          hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  const uint32_t grid = (uint32_t)ncu * (uint32_t)std::min(per_cu, 8);
  j0_kernel<PIPE, LO32><<<grid, CONF_BLOCK, dyn, s>>>(jobs, segs, nseg, tiles);
  return hipGetLastError();
}

hipError_t launch_j0(const Job* jobs, const ConfSeg* segs, int nseg, uint32_t max_points,
                     bool lo32, const uint32_t* tiles, hipStream_t s) {
  if (nseg == 0) return hipSuccess;
  if (lo32 && g_j0_fields == 0)
    return g_j0_variant == 1 ? j0_go<true, true>(jobs, segs, nseg, max_points, tiles, s)
                             : j0_go<false, true>(jobs, segs, nseg, max_points, tiles, s);
  return g_j0_variant == 1 ? j0_go<true, false>(jobs, segs, nseg, max_points, tiles, s)
                           : j0_go<false, false>(jobs, segs, nseg, max_points, tiles, s);
}

hipError_t launch_pairs(const Job* job, rp_pair* out, uint64_t* total, hipStream_t s) {
  pairs_kernel<<<1, 1024, 0, s>>>(job, out, total);
  return hipGetLastError();
}

}  // namespace rp

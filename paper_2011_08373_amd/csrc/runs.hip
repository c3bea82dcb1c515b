// Run log: built once per kernel from the sorted access records.
//
// A run is the set of records of one point at one location (array, word and,
// in the same-block view, block).  Everything a Verify call needs from a run
// is independent of the barrier assignment: its point, whether the point
// writes, whether it holds two or more threads (same-block view) or blocks
// (cross-block view), the id of its first record and whether it opens a new
// location.  The run log stores that in one 64-bit entry per run, in sorted
// order, so every Verify call streams 8 bytes per run instead of rescanning
// the records.
//
//   runs_count_kernel  run heads per tile of 4096 records
//   runs_scan_kernel   per log: exclusive scan of the tile counts, run total
//   runs_write_kernel  per tile: the entries of the runs that start in it
// Records are read coalesced, one per lane; run heads and run ends come from
// 64-lane ballots.
#include "common.h"
#include "launch.h"

namespace rp {

constexpr int RB_BLOCK = 256;
constexpr int RB_WAVES = RB_BLOCK / 64;
constexpr int RB_ROUNDS = 16;                          // block-wide rows of 256 records
constexpr uint32_t RB_TILE = RB_BLOCK * RB_ROUNDS;    // 4096 records

struct ViewBits {
  int psh, lsh, ish;     // point field, location, id shifts
  uint64_t imask;
  uint32_t pmask;
};

__device__ __forceinline__ ViewBits view_bits(const Job& J, uint32_t level) {
  ViewBits v;
  // same-block view: [array|word|block|point|thread]; location = (array, word, block)
  // cross-block view: [array|word|point|block|0];     location = (array, word)
  v.psh = level == 0 ? (int)J.tbits : (int)(J.bbits + J.tbits);
  v.lsh = v.psh + (int)J.pbits;
  v.ish = level == 0 ? 0 : (int)J.tbits;
  v.imask = level == 0 ? ((1ull << J.tbits) - 1) : ((1ull << J.bbits) - 1);
  v.pmask = (1u << J.pbits) - 1u;
  return v;
}

__device__ __forceinline__ int find_seg_by_btile(const ConfSeg* segs, int nseg, uint32_t t) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].btile_beg <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Record q of a log and the one before it (coalesced: lane k reads q0 + k;
// the predecessor comes from the lane below, lane 0 reads it).
__device__ __forceinline__ void rec_and_prev(const uint64_t* log, uint64_t q, uint64_t n,
                                             uint64_t& v, uint64_t& pr) {
  v = q < n ? log[q] : 0;
  pr = __shfl_up(v, 1);
  if (__lane_id() == 0) pr = (q > 0 && q <= n) ? log[q - 1] : 0;
}

__global__ __launch_bounds__(RB_BLOCK) void runs_count_kernel(const Job* __restrict__ jobs,
                                                              const ConfSeg* __restrict__ segs,
                                                              int nseg, uint32_t* __restrict__ cnt) {
  __shared__ uint32_t s_sum[RB_WAVES];
  const uint32_t tile = blockIdx.x;
  const int si = find_seg_by_btile(segs, nseg, tile);
  const ConfSeg& sg = segs[si];
  const ViewBits vb = view_bits(jobs[sg.job], sg.level);
  const uint64_t base = (uint64_t)(tile - sg.btile_beg) * RB_TILE;
  const uint64_t n = sg.n;
  uint32_t c = 0;
  for (int k = 0; k < RB_ROUNDS; k++) {
    const uint64_t q = base + (uint64_t)k * RB_BLOCK + threadIdx.x;
    uint64_t v, pr;
    rec_and_prev(sg.log, q, n, v, pr);
    const bool head = q < n && (q == 0 || (pr >> vb.psh) != (v >> vb.psh));
    c += (uint32_t)__popcll(__ballot(head));
  }
  if (__lane_id() == 0) s_sum[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < RB_WAVES; w++) t += s_sum[w];
    cnt[tile] = t;
  }
}

// One workgroup per log: exclusive scan of its tile counts.
__global__ __launch_bounds__(1024) void runs_scan_kernel(ConfSeg* segs, const uint32_t* __restrict__ cnt,
                                                         uint64_t* __restrict__ off) {
  __shared__ uint64_t sm[16];
  ConfSeg& sg = segs[blockIdx.x];
  const uint32_t t0 = sg.btile_beg;
  const uint32_t nt = (uint32_t)((sg.n + RB_TILE - 1) / RB_TILE);
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  uint64_t run = 0;
  for (uint32_t b = 0; b < nt; b += 1024) {
    const uint32_t t = b + threadIdx.x;
    const uint64_t v = t < nt ? cnt[t0 + t] : 0;
    uint64_t inc = v;
    for (int o = 1; o < 64; o <<= 1) {
      uint64_t y = __shfl_up(inc, o);
      if (lane >= o) inc += y;
    }
    if (lane == 63) sm[w] = inc;
    __syncthreads();
    uint64_t pre = 0, all = 0;
    for (int q = 0; q < 16; q++) {
      if (q < w) pre += sm[q];
      all += sm[q];
    }
    if (t < nt) off[t0 + t] = run + pre + inc - v;
    run += all;
    __syncthreads();
  }
  if (threadIdx.x == 0) sg.n_runs = run;
}

// Entries of the runs that start in one tile.  Rows of 256 consecutive
// records, one per thread, kept in registers across the two passes; a run's
// end is the next head in the wave's 64 records, else it is followed in
// global memory (exponential then binary search for long runs).
__global__ __launch_bounds__(RB_BLOCK) void runs_write_kernel(const Job* __restrict__ jobs,
                                                              const ConfSeg* __restrict__ segs,
                                                              int nseg,
                                                              const uint64_t* __restrict__ off) {
  __shared__ uint32_t s_cnt[RB_ROUNDS * RB_WAVES];
  __shared__ uint64_t s_pre[RB_ROUNDS * RB_WAVES];
  __shared__ uint64_t s_wb[MAX_POINTS / 64];
  const uint32_t tile = blockIdx.x;
  const int si = find_seg_by_btile(segs, nseg, tile);
  const ConfSeg& sg = segs[si];
  const Job& J = jobs[sg.job];
  for (uint32_t q = threadIdx.x; q < (J.P + 63) / 64; q += RB_BLOCK) s_wb[q] = J.wbits[q];
  const ViewBits vb = view_bits(J, sg.level);
  const uint64_t n = sg.n;
  const uint64_t* __restrict__ log = sg.log;
  const uint64_t base = (uint64_t)(tile - sg.btile_beg) * RB_TILE;
  const int lane = __lane_id(), wv = threadIdx.x >> 6;
  uint64_t vv[RB_ROUNDS], pp[RB_ROUNDS], hh[RB_ROUNDS];
  // pass 1: head masks per (row, wave), in record order
#pragma unroll
  for (int k = 0; k < RB_ROUNDS; k++) {
    const uint64_t q = base + (uint64_t)k * RB_BLOCK + threadIdx.x;
    rec_and_prev(log, q, n, vv[k], pp[k]);
    hh[k] = __ballot(q < n && (q == 0 || (pp[k] >> vb.psh) != (vv[k] >> vb.psh)));
    if (lane == 0) s_cnt[k * RB_WAVES + wv] = (uint32_t)__popcll(hh[k]);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = off[tile];
    for (int q = 0; q < RB_ROUNDS * RB_WAVES; q++) {
      s_pre[q] = t;
      t += s_cnt[q];
    }
  }
  __syncthreads();
  // pass 2: entries
#pragma unroll
  for (int k = 0; k < RB_ROUNDS; k++) {
    const uint64_t q = base + (uint64_t)k * RB_BLOCK + threadIdx.x;
    const uint64_t v = vv[k], pr = pp[k], hm = hh[k];
    const bool head = (hm >> lane) & 1;
    const uint64_t above = lane == 63 ? 0ull : (hm >> (lane + 1));
    const int nxt = above ? lane + __ffsll((unsigned long long)above) : 64;   // next head lane
    const uint64_t last_in = __shfl(v, nxt - 1);
    if (!head) continue;
    const uint64_t q_end = q - lane + 64;        // first record past the wave's 64
    uint64_t last, len;
    if (nxt < 64) {                              // ends inside the wave
      last = last_in;
      len = (uint64_t)(nxt - lane);
    } else if (q_end >= n) {                     // ends with the log
      last = log[n - 1];
      len = n - q;
    } else {
      // the run reaches past the wave: find its end in global memory
      const uint64_t pv = v >> vb.psh;
      uint64_t lo = q_end - 1, step = 1, hi;
      for (;;) {
        hi = lo + step;
        if (hi >= n) { hi = n; break; }
        if ((log[hi] >> vb.psh) != pv) break;
        lo = hi;
        step <<= 1;
      }
      while (hi - lo > 1) {
        const uint64_t mid = lo + ((hi - lo) >> 1);
        if ((log[mid] >> vb.psh) == pv) lo = mid; else hi = mid;
      }
      last = log[hi - 1];
      len = hi - q;
    }
    const uint64_t id = (v >> vb.ish) & vb.imask;
    const bool multi = sg.level == 0 ? len >= 2 : ((last >> vb.ish) & vb.imask) != id;
    const bool locstart = q == 0 || (pr >> vb.lsh) != (v >> vb.lsh);
    const uint32_t i = (uint32_t)(v >> vb.psh) & vb.pmask;
    const bool wr = i < J.P && ((s_wb[i >> 6] >> (i & 63)) & 1);
    const uint64_t idx = s_pre[k * RB_WAVES + wv] + (uint64_t)__popcll(hm & lanemask_lt());
    sg.runs[idx] = id | ((uint64_t)i << RUN_PT) | ((uint64_t)wr << RUN_W) |
                   ((uint64_t)multi << RUN_MULTI) | ((uint64_t)locstart << RUN_LOC);
  }
}

uint32_t runs_tile_size() { return RB_TILE; }

hipError_t launch_runs_build(const Job* jobs, ConfSeg* segs, int nseg, uint32_t n_btiles,
                             uint32_t* cnt, uint64_t* off, hipStream_t s) {
  if (nseg == 0 || n_btiles == 0) return hipSuccess;
  runs_count_kernel<<<n_btiles, RB_BLOCK, 0, s>>>(jobs, segs, nseg, cnt);
  runs_scan_kernel<<<nseg, 1024, 0, s>>>(segs, cnt, off);
  runs_write_kernel<<<n_btiles, RB_BLOCK, 0, s>>>(jobs, segs, nseg, off);
  return hipGetLastError();
}

}  // namespace rp

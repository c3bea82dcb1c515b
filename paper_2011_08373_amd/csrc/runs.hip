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
#include "common.h"
#include "launch.h"

namespace rp {

constexpr int RB_BLOCK = 256;
constexpr int RB_PER = 16;                             // contiguous records per thread
constexpr uint32_t RB_TILE = RB_BLOCK * RB_PER;       // 4096 records
constexpr uint32_t RB_LOOK = 1024;                     // staged past the tile
constexpr uint32_t RB_WIN = RB_TILE + RB_LOOK;

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

__global__ __launch_bounds__(RB_BLOCK) void runs_count_kernel(const Job* __restrict__ jobs,
                                                              const ConfSeg* __restrict__ segs,
                                                              int nseg, uint32_t* __restrict__ cnt) {
  __shared__ uint64_t s_rec[RB_TILE];
  __shared__ uint32_t s_sum[RB_BLOCK / 64];
  const uint32_t tile = blockIdx.x;
  const int si = find_seg_by_btile(segs, nseg, tile);
  const ConfSeg sg = segs[si];
  const ViewBits vb = view_bits(jobs[sg.job], sg.level);
  const uint64_t base = (uint64_t)(tile - sg.btile_beg) * RB_TILE;
  const uint32_t len = (uint32_t)((sg.n - base) < RB_TILE ? (sg.n - base) : RB_TILE);
  for (uint32_t q = threadIdx.x; q < len; q += RB_BLOCK) s_rec[q] = sg.log[base + q];
  const uint64_t prev = base > 0 ? sg.log[base - 1] : 0;
  __syncthreads();
  uint32_t c = 0;
  for (uint32_t q = 0; q < RB_PER; q++) {
    const uint32_t p = threadIdx.x * RB_PER + q;
    if (p >= len) break;
    const uint64_t v = s_rec[p];
    if (p == 0 && base == 0) { c++; continue; }
    const uint64_t pr = p ? s_rec[p - 1] : prev;
    if ((pr >> vb.psh) != (v >> vb.psh)) c++;
  }
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if (__lane_id() == 0) s_sum[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) cnt[tile] = s_sum[0] + s_sum[1] + s_sum[2] + s_sum[3];
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

__global__ __launch_bounds__(RB_BLOCK) void runs_write_kernel(const Job* __restrict__ jobs,
                                                              const ConfSeg* __restrict__ segs,
                                                              int nseg,
                                                              const uint64_t* __restrict__ off) {
  __shared__ uint64_t s_rec[RB_WIN];
  __shared__ uint32_t s_head[RB_WIN / 32];
  __shared__ uint32_t s_sum[RB_BLOCK / 64];
  __shared__ uint64_t s_prev;
  const uint32_t tile = blockIdx.x;
  const int si = find_seg_by_btile(segs, nseg, tile);
  const ConfSeg sg = segs[si];
  const Job& J = jobs[sg.job];
  const ViewBits vb = view_bits(J, sg.level);
  const uint64_t n = sg.n;
  const uint64_t base = (uint64_t)(tile - sg.btile_beg) * RB_TILE;
  const uint32_t wlen = (uint32_t)((n - base) < RB_WIN ? (n - base) : RB_WIN);
  const uint32_t own = wlen < RB_TILE ? wlen : RB_TILE;
  for (uint32_t q = threadIdx.x; q < wlen; q += RB_BLOCK) s_rec[q] = sg.log[base + q];
  for (uint32_t q = threadIdx.x; q < RB_WIN / 32; q += RB_BLOCK) s_head[q] = 0;
  if (threadIdx.x == 0) s_prev = base > 0 ? sg.log[base - 1] : 0;
  __syncthreads();
  // head bits over the whole window
  for (uint32_t p = threadIdx.x; p < wlen; p += RB_BLOCK) {
    bool h;
    if (p == 0) h = base == 0 || (s_prev >> vb.psh) != (s_rec[0] >> vb.psh);
    else h = (s_rec[p - 1] >> vb.psh) != (s_rec[p] >> vb.psh);
    if (h) atomicOr(&s_head[p >> 5], 1u << (p & 31));
  }
  __syncthreads();
  // ranks of the owned heads (contiguous positions per thread keep run order)
  const uint32_t p0 = threadIdx.x * RB_PER;
  uint32_t mine = 0;
  for (uint32_t q = 0; q < RB_PER; q++) {
    const uint32_t p = p0 + q;
    if (p < own && ((s_head[p >> 5] >> (p & 31)) & 1)) mine++;
  }
  uint32_t inc = mine;
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == 63) s_sum[w] = inc;
  __syncthreads();
  uint32_t pre = 0;
  for (int q = 0; q < w; q++) pre += s_sum[q];
  uint64_t idx = off[tile] + pre + inc - mine;
  for (uint32_t q = 0; q < RB_PER; q++) {
    const uint32_t p = p0 + q;
    if (p >= own || !((s_head[p >> 5] >> (p & 31)) & 1)) continue;
    const uint64_t v = s_rec[p];
    // run end: the next head in the window, else past it
    uint32_t e = p + 1;
    while (e < wlen && !((s_head[e >> 5] >> (e & 31)) & 1)) {
      if ((e & 31) == 0 && s_head[e >> 5] == 0) { e += 32; continue; }
      e++;
    }
    uint64_t last;
    uint64_t glen;   // run length, exact when it ends inside the window
    if (e < wlen || base + wlen == n) {
      if (e > wlen) e = wlen;
      last = s_rec[e - 1];
      glen = e - p;
    } else {
      // the run continues past the window: find its end in global memory
      const uint64_t pv = v >> vb.psh;
      uint64_t lo = base + wlen - 1, step = 1, hi;
      for (;;) {
        hi = lo + step;
        if (hi >= n) { hi = n; break; }
        if ((sg.log[hi] >> vb.psh) != pv) break;
        lo = hi;
        step <<= 1;
      }
      while (hi - lo > 1) {
        const uint64_t mid = lo + ((hi - lo) >> 1);
        if ((sg.log[mid] >> vb.psh) == pv) lo = mid; else hi = mid;
      }
      last = sg.log[hi - 1];
      glen = hi - (base + p);
    }
    const uint64_t id = (v >> vb.ish) & vb.imask;
    const bool multi = sg.level == 0 ? glen >= 2 : ((last >> vb.ish) & vb.imask) != id;
    const uint64_t prv = p ? s_rec[p - 1] : s_prev;
    const bool locstart = (p == 0 && base == 0) || (prv >> vb.lsh) != (v >> vb.lsh);
    const uint32_t i = (uint32_t)(v >> vb.psh) & vb.pmask;
    const bool wr = i < J.P && (J.pts[i].flags & PF_WRITE);
    sg.runs[idx++] = id | ((uint64_t)i << RUN_PT) | ((uint64_t)wr << RUN_W) |
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

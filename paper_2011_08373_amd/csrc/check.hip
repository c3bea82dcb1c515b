// Verify under an assignment x (the concrete counterpart of the verifier call
// of Alg. 1).
//
// ivl_kernel   one workgroup per job: interval ids = number of enabled
//              barrier occurrences before each point (any level, and grid
//              level only), the divergent enabled slots, and the reset of the
//              per-round outputs.
// conf_kernel  scan of the run logs (runs.hip).  Runs are in program order
//              inside a location, so the runs of one interval are contiguous.
//              Two runs race when one writes and they are not the same single
//              thread (same-block view) or the same single block (cross-block
//              view).  In "first" mode a run stops at its first racing
//              partner (enough for the reduced clause set); in "all" mode
//              every racing pair goes into a bitmap.
// pairs_kernel turns the bitmap into the (level, i, j)-ordered pair list.
#include "common.h"
#include "launch.h"

namespace rp {

constexpr int IVL_BLOCK = 1024;
constexpr int CONF_BLOCK = 256;
constexpr uint32_t CONF_TILE = 4096;                     // runs owned per tile
constexpr uint32_t CONF_WIN = CONF_TILE + 2048;          // staged: tile + lookahead

__global__ __launch_bounds__(IVL_BLOCK) void ivl_kernel(const Job* __restrict__ jobs, int with_bitmap) {
  __shared__ uint64_t wsum[IVL_BLOCK / 64];
  const Job& J = jobs[blockIdx.x];
  JobState* st = J.st;
  if (st->state != ST_RUN) return;
  const uint64_t x = st->x;
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
      J.ivl[i] = (uint32_t)run;               // enabled occurrences before i
      J.ivl[P + i] = (uint32_t)(run >> 32);   // enabled GRID occurrences before i
    }
    run += cnt[q];
  }
  for (uint32_t i = tid; i < 2 * P; i += IVL_BLOCK) J.minj[i] = NONE32;
  if (with_bitmap && J.bitmap) {
    const uint64_t nw = 2ull * P * J.wpr;
    for (uint64_t q = tid; q < nw; q += IVL_BLOCK) J.bitmap[q] = 0;
  }
  if (tid == 0) st->divergent = x & J.div_if_enabled;
}

__device__ __forceinline__ void set_pair(uint64_t* bm, uint32_t wpr, uint32_t P, uint32_t lv,
                                         uint32_t i, uint32_t j) {
  uint64_t* wp = bm + ((uint64_t)lv * P + i) * wpr + (j >> 6);
  const uint64_t bit = 1ull << (j & 63);
  if (!(*wp & bit)) atomicOr((unsigned long long*)wp, (unsigned long long)bit);
}

// Racing partners over the run log.  A sub-segment (one location, one
// interval) is a contiguous stretch of runs; each run looks at the runs after
// it in its sub-segment.  Tiles of runs plus a lookahead are staged in LDS,
// reads past the staged window go to global memory.
__global__ __launch_bounds__(CONF_BLOCK) void conf_kernel(const Job* __restrict__ jobs,
                                                          const ConfSeg* __restrict__ segs,
                                                          int nseg, uint32_t n_tiles,
                                                          uint32_t tiles_per_wg, int all_pairs) {
  __shared__ uint64_t s_run[CONF_WIN];
  extern __shared__ uint32_t s_dyn[];        // [P] interval of each point, [P] first partner
  const int tid = threadIdx.x;
  const uint32_t t0 = blockIdx.x * tiles_per_wg;
  uint32_t t1 = t0 + tiles_per_wg;
  if (t1 > n_tiles) t1 = n_tiles;
  int cur = -1;
  bool live = false;
  uint32_t* s_iv = s_dyn;
  uint32_t* s_minj = s_dyn;   // placed after s_iv once P is known
  for (uint32_t tile = t0; tile < t1; tile++) {
    int lo = 0, hi = nseg - 1;   // largest segment with ctile_beg <= tile
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (segs[mid].ctile_beg <= tile) lo = mid; else hi = mid - 1;
    }
    if (lo != cur) {
      if (cur >= 0 && live && !all_pairs) {
        __syncthreads();
        const Job& J = jobs[segs[cur].job];
        uint32_t* g = J.minj + (uint64_t)segs[cur].level * J.P;
        for (uint32_t i = tid; i < J.P; i += CONF_BLOCK)
          if (s_minj[i] != NONE32) atomicMin(&g[i], s_minj[i]);
      }
      __syncthreads();
      cur = lo;
      const Job& J = jobs[segs[cur].job];
      s_minj = s_dyn + J.P;
      live = J.st->state == ST_RUN;
      if (live) {
        const uint32_t* iv = J.ivl + (uint64_t)segs[cur].level * J.P;
        for (uint32_t i = tid; i < J.P; i += CONF_BLOCK) {
          s_iv[i] = iv[i];
          s_minj[i] = NONE32;
        }
      }
      __syncthreads();
    }
    if (!live) continue;
    const ConfSeg sg = segs[cur];
    const uint64_t n = sg.n_runs_at ? *sg.n_runs_at : sg.n_runs;
    const uint64_t base = (uint64_t)(tile - sg.ctile_beg) * CONF_TILE;
    if (base >= n) continue;   // run counts are known on the device only
    const Job& J = jobs[sg.job];
    const uint32_t P = J.P;
    const uint64_t* __restrict__ runs = sg.runs;
    const uint32_t wlen = (uint32_t)((n - base) < CONF_WIN ? (n - base) : CONF_WIN);
    const uint32_t own = wlen < CONF_TILE ? wlen : CONF_TILE;
    __syncthreads();
    for (uint32_t q = tid; q < wlen; q += CONF_BLOCK) s_run[q] = runs[base + q];
    __syncthreads();
    for (uint32_t r = tid; r < own; r += CONF_BLOCK) {
      const uint64_t ei = s_run[r];
      const uint32_t i = (uint32_t)(ei >> RUN_PT) & 0xFFFu;
      if (i >= P) continue;
      const bool wi = (ei >> RUN_W) & 1, mi = (ei >> RUN_MULTI) & 1;
      const uint32_t idi = (uint32_t)ei, iv = s_iv[i];
      if (wi && mi) {
        if (all_pairs) set_pair(J.bitmap, J.wpr, P, sg.level, i, i);
        else { atomicMin(&s_minj[i], i); continue; }
      }
      for (uint64_t q = base + r + 1; q < n; q++) {
        const uint64_t ej = (q - base) < wlen ? s_run[q - base] : runs[q];
        if ((ej >> RUN_LOC) & 1) break;             // next location
        const uint32_t j = (uint32_t)(ej >> RUN_PT) & 0xFFFu;
        if (j >= P || s_iv[j] != iv) break;          // next interval
        if ((wi || ((ej >> RUN_W) & 1)) && (mi || ((ej >> RUN_MULTI) & 1) || idi != (uint32_t)ej)) {
          if (all_pairs) {
            set_pair(J.bitmap, J.wpr, P, sg.level, i, j);
          } else {
            atomicMin(&s_minj[i], j);
            break;
          }
        }
      }
    }
  }
  if (cur >= 0 && live && !all_pairs) {
    __syncthreads();
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

hipError_t launch_ivl(const Job* jobs, uint32_t njobs, int with_bitmap, hipStream_t s) {
  if (njobs == 0) return hipSuccess;
  ivl_kernel<<<njobs, IVL_BLOCK, 0, s>>>(jobs, with_bitmap);
  return hipGetLastError();
}

hipError_t launch_conf(const Job* jobs, const ConfSeg* segs, int nseg, uint32_t n_tiles,
                       uint32_t grid, uint32_t max_points, int all_pairs, hipStream_t s) {
  if (n_tiles == 0 || nseg == 0) return hipSuccess;
  if (grid > n_tiles) grid = n_tiles;
  const uint32_t per = (n_tiles + grid - 1) / grid;
  grid = (n_tiles + per - 1) / per;
  const size_t dyn = 2 * (size_t)(max_points ? max_points : 1) * sizeof(uint32_t);
  conf_kernel<<<grid, CONF_BLOCK, dyn, s>>>(jobs, segs, nseg, n_tiles, per, all_pairs);
  return hipGetLastError();
}

hipError_t launch_pairs(const Job* job, rp_pair* out, uint64_t* total, hipStream_t s) {
  pairs_kernel<<<1, 1024, 0, s>>>(job, out, total);
  return hipGetLastError();
}

}  // namespace rp

// Verify under an assignment x (the concrete counterpart of the verifier call
// of Alg. 1).
//
// ivl_kernel   one workgroup per job: interval ids = number of enabled
//              barrier occurrences before each point (any level, and grid
//              level only), the divergent enabled slots, and the reset of the
//              per-round outputs.
// conf_kernel  persistent scan of the sorted logs.  A "run" is the records of
//              one point at one location; runs are in program order inside a
//              location, so the runs of one interval are contiguous.  Each run
//              head walks the following runs of its location and interval and
//              reports racing partners: two runs race when one writes and they
//              are not the same single thread (same-block view) or the same
//              single block (cross-block view).  In "first" mode a run stops
//              at its first racing partner (enough for the reduced clause set);
//              in "all" mode every racing pair goes into a bitmap.
// pairs_kernel turns the bitmap into the (level, i, j)-ordered pair list.
#include "common.h"
#include "launch.h"

namespace rp {

constexpr int IVL_BLOCK = 1024;
constexpr int CONF_BLOCK = 256;
constexpr uint32_t CONF_TILE = 2048;                     // records owned per tile
constexpr uint32_t CONF_WIN = CONF_TILE + 1024;          // staged: tile + lookahead

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

// The records of one tile plus a lookahead are staged in LDS; reads past
// the staged window fall back to global memory.
struct Win {
  const uint64_t* __restrict__ g;
  const uint64_t* s;
  uint64_t base, len;
  __device__ __forceinline__ uint64_t operator()(uint64_t i) const {
    const uint64_t o = i - base;   // callers never read below base
    return o < len ? s[o] : g[i];
  }
};

// First index after q whose (location, point) prefix differs from pv.
__device__ __forceinline__ uint64_t run_end(const Win& at, uint64_t n, uint64_t q, uint64_t pv,
                                            int psh) {
  uint64_t lo = q + 1;
  if (lo >= n || (at(lo) >> psh) != pv) return lo;
  uint64_t step = 1, hi;
  for (;;) {
    hi = lo + step;
    if (hi >= n) { hi = n; break; }
    if ((at(hi) >> psh) != pv) break;
    lo = hi;
    step <<= 1;
  }
  while (hi - lo > 1) {
    const uint64_t mid = lo + ((hi - lo) >> 1);
    if ((at(mid) >> psh) == pv) lo = mid; else hi = mid;
  }
  return hi;
}

__device__ __forceinline__ void set_pair(uint64_t* bm, uint32_t wpr, uint32_t P, uint32_t lv,
                                         uint32_t i, uint32_t j) {
  uint64_t* wp = bm + ((uint64_t)lv * P + i) * wpr + (j >> 6);
  const uint64_t bit = 1ull << (j & 63);
  if (!(*wp & bit)) atomicOr((unsigned long long*)wp, (unsigned long long)bit);
}

// run-table entry: id | point << 32 | write << 44 | multi << 45 | sub << 47
constexpr int RT_PT = 32, RT_W = 44, RT_MULTI = 45, RT_SUB = 47;

__device__ __forceinline__ uint64_t block_excl_scan256_u64(uint64_t v, uint64_t* sm,
                                                          uint64_t* total) {
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  uint64_t inc = v;
  for (int o = 1; o < 64; o <<= 1) {
    uint64_t y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == 63) sm[w] = inc;
  __syncthreads();
  uint64_t pre = 0, tot = 0;
  for (int q = 0; q < CONF_BLOCK / 64; q++) {
    if (q < w) pre += sm[q];
    tot += sm[q];
  }
  __syncthreads();
  *total = tot;
  return pre + inc - v;
}

__global__ __launch_bounds__(CONF_BLOCK) void conf_kernel(const Job* __restrict__ jobs,
                                                          const ConfSeg* __restrict__ segs,
                                                          int nseg, uint32_t n_tiles,
                                                          uint32_t tiles_per_wg, int all_pairs) {
  __shared__ uint64_t s_rec[CONF_WIN];        // records of the tile and the lookahead
  __shared__ uint64_t s_info[CONF_WIN];       // run table
  __shared__ uint16_t s_rstart[CONF_WIN + 1]; // run start positions in the window
  __shared__ uint64_t s_sm[CONF_BLOCK / 64];
  __shared__ uint64_t s_prev;
  extern __shared__ uint32_t s_dyn[];         // [P] (interval << 1) | write, [P] first partner
  const int tid = threadIdx.x;
  const uint32_t t0 = blockIdx.x * tiles_per_wg;
  uint32_t t1 = t0 + tiles_per_wg;
  if (t1 > n_tiles) t1 = n_tiles;
  int cur = -1;
  bool live = false;
  uint32_t* s_pt = s_dyn;
  uint32_t* s_minj = s_dyn;   // placed after s_pt once P is known
  for (uint32_t tile = t0; tile < t1; tile++) {
    int lo = 0, hi = nseg - 1;   // largest segment with tile_beg <= tile
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (segs[mid].tile_beg <= tile) lo = mid; else hi = mid - 1;
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
          s_pt[i] = (iv[i] << 1) | ((J.pts[i].flags & PF_WRITE) ? 1u : 0u);
          s_minj[i] = NONE32;
        }
      }
      __syncthreads();
    }
    if (!live) continue;
    const ConfSeg sg = segs[cur];
    const Job& J = jobs[sg.job];
    const uint32_t P = J.P;
    const uint64_t* __restrict__ log = sg.log;
    const uint64_t n = sg.n;
    const uint64_t base = (uint64_t)(tile - sg.tile_beg) * CONF_TILE;
    const uint32_t wlen = (uint32_t)((n - base) < CONF_WIN ? (n - base) : CONF_WIN);
    const bool at_end = base + wlen == n;
    const uint32_t tb = J.tbits, bb = J.bbits, pb = J.pbits;
    const uint32_t pmask = (1u << pb) - 1u;
    // same-block view: location = (array, word, block), id = thread
    // cross-block view: location = (array, word), id = block
    const int psh = sg.level == 0 ? (int)tb : (int)(bb + tb);
    const int lsh = psh + (int)pb;
    const int ish = sg.level == 0 ? 0 : (int)tb;
    const uint64_t imask = sg.level == 0 ? ((1ull << tb) - 1) : ((1ull << bb) - 1);
    __syncthreads();
    for (uint32_t q = tid; q < wlen; q += CONF_BLOCK) s_rec[q] = log[base + q];
    if (tid == 0) s_prev = base > 0 ? log[base - 1] : 0;
    __syncthreads();

    // ---- 1. run heads and sub-segment starts (contiguous positions per thread)
    constexpr uint32_t PER = CONF_WIN / CONF_BLOCK;
    const uint32_t p0 = tid * PER;
    uint32_t hmask = 0, smask = 0;
    for (uint32_t q = 0; q < PER; q++) {
      const uint32_t p = p0 + q;
      if (p >= wlen) break;
      const uint64_t v = s_rec[p];
      const bool has_prev = p > 0 || base > 0;
      if (!has_prev) { hmask |= 1u << q; smask |= 1u << q; continue; }
      const uint64_t pr = p > 0 ? s_rec[p - 1] : s_prev;
      if ((pr >> psh) == (v >> psh)) continue;
      hmask |= 1u << q;
      const uint32_t i = (uint32_t)(v >> psh) & pmask, ip = (uint32_t)(pr >> psh) & pmask;
      if ((pr >> lsh) != (v >> lsh) || i >= P || ip >= P || (s_pt[i] >> 1) != (s_pt[ip] >> 1))
        smask |= 1u << q;
    }
    uint64_t tot;
    const uint64_t ex = block_excl_scan256_u64(((uint64_t)__popc(smask) << 32) | __popc(hmask),
                                               s_sm, &tot);
    const uint32_t n_runs = (uint32_t)tot;
    uint32_t ri = (uint32_t)ex, sub = (uint32_t)(ex >> 32);
    for (uint32_t q = 0; q < PER; q++) {
      if (!((hmask >> q) & 1)) continue;
      const uint32_t p = p0 + q;
      sub += (smask >> q) & 1;
      const uint64_t v = s_rec[p];
      const uint32_t i = (uint32_t)(v >> psh) & pmask;
      const uint64_t w = (i < P) ? (uint64_t)(s_pt[i] & 1) : 0;
      s_rstart[ri] = (uint16_t)p;
      s_info[ri] = ((v >> ish) & imask) | ((uint64_t)i << RT_PT) | (w << RT_W) |
                   ((uint64_t)sub << RT_SUB);
      ri++;
    }
    if (tid == 0) s_rstart[n_runs] = (uint16_t)wlen;
    __syncthreads();

    // ---- 2. multiplicity (two threads, or two blocks, in the run)
    for (uint32_t r = tid; r < n_runs; r += CONF_BLOCK) {
      const uint32_t st = s_rstart[r], en = s_rstart[r + 1];
      const bool open = r + 1 == n_runs && !at_end;
      const uint64_t first = s_rec[st];
      bool multi;
      if (sg.level == 0) {
        multi = en - st >= 2;
        if (!multi && open) multi = (log[base + wlen] >> psh) == (first >> psh);
      } else {
        const uint64_t oid = (first >> ish) & imask;
        multi = ((s_rec[en - 1] >> ish) & imask) != oid;
        if (!multi && open) {
          const Win at{log, s_rec, base, wlen};
          const uint64_t e = run_end(at, n, base + en - 1, first >> psh, psh);
          multi = ((log[e - 1] >> ish) & imask) != oid;
        }
      }
      if (multi) s_info[r] |= 1ull << RT_MULTI;
    }
    __syncthreads();

    // ---- 3. partners of the runs that start in this tile
    const uint32_t own = wlen < CONF_TILE ? wlen : CONF_TILE;
    for (uint32_t r = tid; r < n_runs; r += CONF_BLOCK) {
      const uint32_t st = s_rstart[r];
      if (st >= own) break;
      const uint64_t ei = s_info[r];
      const uint32_t i = (uint32_t)(ei >> RT_PT) & 0xFFFu;
      if (i >= P) continue;
      const bool wi = (ei >> RT_W) & 1, mi = (ei >> RT_MULTI) & 1;
      const uint32_t idi = (uint32_t)ei, subi = (uint32_t)(ei >> RT_SUB);
      if (wi && mi) {
        if (all_pairs) set_pair(J.bitmap, J.wpr, P, sg.level, i, i);
        else { atomicMin(&s_minj[i], i); continue; }
      }
      bool done = false;
      uint32_t rj = r + 1;
      for (; rj < n_runs; rj++) {
        const uint64_t ej = s_info[rj];
        if ((uint32_t)(ej >> RT_SUB) != subi) { done = true; break; }
        const uint32_t j = (uint32_t)(ej >> RT_PT) & 0xFFFu;
        if (j >= P) continue;
        if ((wi || ((ej >> RT_W) & 1)) && (mi || ((ej >> RT_MULTI) & 1) || idi != (uint32_t)ej)) {
          if (all_pairs) {
            set_pair(J.bitmap, J.wpr, P, sg.level, i, j);
          } else {
            atomicMin(&s_minj[i], j);
            done = true;
            break;
          }
        }
      }
      if (done || at_end) continue;
      // the sub-segment may continue past the window: walk on in global memory
      const Win at{log, s_rec, base, wlen};
      const uint64_t v = s_rec[st];
      const uint64_t loc = v >> lsh;
      const uint32_t iv = s_pt[i] >> 1;
      uint64_t q;
      {
        const uint32_t lr = n_runs - 1;   // last run of the window, maybe open
        const uint64_t lv = s_rec[s_rstart[lr]];
        q = run_end(at, n, base + s_rstart[lr], lv >> psh, psh);
      }
      while (q < n) {
        const uint64_t vq = at(q);
        if ((vq >> lsh) != loc) break;
        const uint64_t pq = vq >> psh;
        const uint32_t j = (uint32_t)pq & pmask;
        if (j >= P) break;
        const uint32_t jpt = s_pt[j];
        if ((jpt >> 1) != iv) break;
        const uint64_t eq = run_end(at, n, q, pq, psh);
        if (wi || (jpt & 1)) {
          const uint64_t jid = (vq >> ish) & imask;
          const bool jmulti = sg.level == 0 ? (eq - q >= 2) : (((at(eq - 1) >> ish) & imask) != jid);
          if (mi || jmulti || (uint64_t)idi != jid) {
            if (all_pairs) {
              set_pair(J.bitmap, J.wpr, P, sg.level, i, j);
            } else {
              atomicMin(&s_minj[i], j);
              break;
            }
          }
        }
        q = eq;
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

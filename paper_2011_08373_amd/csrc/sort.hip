// Stable LSD radix sort of the access records (reduce-then-scan per pass).
//
// The record buffer is cut into chunks that never straddle a sort segment
// (one log of one job).  Per digit pass:
//   count_kernel     per chunk, how many records carry each digit, read
//                    from the digit array the previous pass's scatter wrote
//                    beside its output (1 byte per record for 8-bit digits,
//                    2 above), not from the 8-byte records (pass 0 takes its
//                    counts from record generation instead);
//   colpart/coltot/colbase(_small)/coloff_kernel
//                    the exclusive scan of the counts per (segment, digit)
//                    over the chunks, offset by the segment start and the
//                    totals of smaller digits: the first output slot of
//                    every (chunk, digit);
//   scatter_kernel   per chunk, tiles of records are ranked stably with
//                    64-lane ballots, staged in LDS in digit order and written
//                    out as contiguous digit runs, each record's digit of the
//                    next pass beside it in the digit array; a persistent grid sized to
//                    the resident workgroups takes chunks from a ticket
//                    counter (reset by the column scan of the same pass), so
//                    equal chunks that do not divide evenly among the
//                    workgroups leave no idle tail.
// No workgroup ever waits on another (a ticket is one atomic add), so nothing
// here can stall the grid.
#include <algorithm>
#include <type_traits>

#include "common.h"
#include "launch.h"

namespace rp {

constexpr uint32_t SC_MAX_TILE = 8192;   // chunks are multiples of every tile shape

// Digit of the next pass as stored by the scatter: one byte for 8-bit
// digits, two for wider ones.
template <int RB>
using DigT = typename std::conditional<(RB <= 8), uint8_t, uint16_t>::type;

// Per-chunk digit counts of one pass: cnt[chunk][d], from the digit array
// (digit of record q at dig[q]).  The chunk is read in rows of 64 16-byte
// vectors (V = 16 or 8 digits per lane), one row per load instruction, so
// each load takes whole lines and no line is fetched twice; wave w of the
// workgroup takes rows w, w + 4, ... with CNT_U rows in flight per lane and
// the next CNT_U issued before the current ones are counted.  A lane holds
// V consecutive records and merges each run of one digit into a single LDS
// add of the run's length (runs are long where consecutive threads touch
// consecutive words).  Lanes of one add that hit the same counter are served
// one after another, so the lanes count into G copies of the histogram,
// chosen so that lanes sharing a digit in the two common patterns sit in
// different copies: runs put neighbouring lanes on one digit, and a digit
// that rises by one per record puts lane l on digit l * V + k (mod R), so
// lanes R / V apart share it when R / V < 64.  Hence one copy per lane up to
// 7-bit digits, lane / 4 for 8-bit ones (16 copies; lanes 16 apart share a
// digit), lane mod G for wider ones (no two lanes of a row share a rising
// digit).  Copies are R + 1 words apart, so the copies of one digit lie in
// different banks.  Digits of the chunk's first and last vectors that lie
// outside it count nothing.
template <int RB>
struct CntCopies {
  static constexpr uint32_t G = RB <= 7 ? 64 : RB == 8 ? 16 : RB <= 10 ? 8 : 4;
  __device__ static uint32_t of(uint32_t lane) {
    return RB <= 7 ? lane : RB == 8 ? (lane >> 2) : (lane & (G - 1));
  }
};
constexpr int CNT_U = 4;
constexpr int CNT_WAVES = 4;

template <int RB>
__global__ __launch_bounds__(64 * CNT_WAVES) void count_kernel(const DigT<RB>* __restrict__ dig,
                                                               const SortChunk* __restrict__ chunks,
                                                               uint32_t nchunks,
                                                               uint32_t* __restrict__ cnt) {
  constexpr uint32_t R = 1u << RB;
  using D = DigT<RB>;
  constexpr uint32_t V = 16 / sizeof(D);          // digits per vector
  constexpr uint32_t G = CntCopies<RB>::G;
  constexpr uint32_t HS = R + 1;                 // copy stride: copies of a digit a bank apart
  constexpr uint32_t NT = 64 * CNT_WAVES;
  __shared__ uint32_t hist[G * HS];
  const uint32_t tid = threadIdx.x, lane = __lane_id();
  const uint32_t w = __builtin_amdgcn_readfirstlane(tid >> 6);
  uint32_t* my = hist + CntCopies<RB>::of(lane) * HS;
  const uint4* src = reinterpret_cast<const uint4*>(dig);
  for (uint32_t ci = blockIdx.x; ci < nchunks; ci += gridDim.x) {   // persistent
    const SortChunk ch = chunks[ci];
    __syncthreads();
    for (uint32_t d = tid; d < G * HS; d += NT) hist[d] = 0;
    __syncthreads();
    // vectors covering [beg, end), aligned to V digits, in rows of 64
    const uint64_t v0 = ch.beg / V, v1 = (ch.end + V - 1) / V;
    const uint64_t nrow = (v1 - v0 + 63) / 64;
    // loads past the chunk read its last vector (always in bounds, so no
    // load is conditional) and count nothing
    const uint64_t vlast = v1 - 1;
    auto row_vec = [&](uint64_t r) { return v0 + r * 64 + lane; };
    uint4 cur[CNT_U];
    uint64_t r = w;
#pragma unroll
    for (int u = 0; u < CNT_U; u++) {
      const uint64_t v = row_vec(r + (uint64_t)u * CNT_WAVES);
      cur[u] = src[v < v1 ? v : vlast];
    }
    for (; r < nrow; r += (uint64_t)CNT_U * CNT_WAVES) {
      const uint64_t rn = r + (uint64_t)CNT_U * CNT_WAVES;
      uint4 nxt[CNT_U];
#pragma unroll
      for (int u = 0; u < CNT_U; u++) {
        const uint64_t v = row_vec(rn + (uint64_t)u * CNT_WAVES);
        nxt[u] = src[v < v1 ? v : vlast];
      }
#pragma unroll
      for (int u = 0; u < CNT_U; u++) {
        const D* e = reinterpret_cast<const D*>(&cur[u]);
        const uint64_t v = row_vec(r + (uint64_t)u * CNT_WAVES);
        const uint64_t q0 = v * V;
        // digits [lo, hi) of this vector lie in the chunk (none past its end)
        const uint32_t lo = q0 >= ch.beg ? 0u : (uint32_t)min((uint64_t)V, ch.beg - q0);
        const uint32_t hi = v >= v1 ? 0u
                            : (q0 + V <= ch.end ? V : (uint32_t)(ch.end > q0 ? ch.end - q0 : 0));
        uint32_t run = 0;
#pragma unroll
        for (uint32_t k = 0; k < V; k++) {
          run += (k - lo < hi - lo) ? 1u : 0u;
          // the run ends at the vector's last digit or before another digit
          const bool ends = k + 1 == V || e[k + 1] != e[k];
          if (ends && run != 0) {
            atomicAdd(&my[e[k]], run);
            run = 0;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < CNT_U; u++) cur[u] = nxt[u];
    }
    __syncthreads();
    uint32_t* row = cnt + (size_t)ci * R;
    for (uint32_t d = tid; d < R; d += NT) {
      uint32_t t = 0;
#pragma unroll 8
      for (uint32_t g = 0; g < G; g++) t += hist[g * HS + d];
      row[d] = t;
    }
  }
}

// Column scans of a pass: off[c][d] = the segment's start + the records of
// smaller digits in the segment + the records of digit d in the segment's
// chunks before c.  The chunks of a segment form column blocks of
// COL_BLOCK_CHUNKS chunks; every table row (one chunk, all digits) is read
// or written whole by a workgroup, one digit per thread.
//   colpart_kernel  per column block and digit, its count (part);
//   coltot_kernel   per segment and digit, the total over its blocks (tot);
//   colbase_kernel  per segment and digit, each block's base: the segment's
//                   start, the smaller digits' totals and the counts of the
//                   blocks before it (part, in place);
//   coloff_kernel   per chunk and digit, the block's base plus the counts of
//                   the block's chunks before it (off).

// The column block's segment (the last with cblk_beg <= b) and chunks.
__device__ __forceinline__ uint32_t cblk_seg(const SortSeg* segs, uint32_t nseg, uint32_t b) {
  uint32_t lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (segs[mid].cblk_beg <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

constexpr int COL_U = 8;   // table loads in flight per thread

template <int RB>
__global__ __launch_bounds__(256) void colpart_kernel(const uint32_t* __restrict__ cnt,
                                                      const SortSeg* __restrict__ segs,
                                                      uint32_t nseg, uint64_t* __restrict__ part) {
  constexpr uint32_t R = 1u << RB;
  const uint32_t b = blockIdx.x;
  const SortSeg sg = segs[cblk_seg(segs, nseg, b)];
  const uint32_t c0 = sg.chunk_beg + (b - sg.cblk_beg) * COL_BLOCK_CHUNKS;
  const uint32_t c1 = min(c0 + COL_BLOCK_CHUNKS, sg.chunk_end);
  for (uint32_t d = threadIdx.x; d < R; d += 256) {
    uint64_t t = 0;
    for (uint32_t c = c0; c < c1; c += COL_U) {
      uint32_t v[COL_U];
#pragma unroll
      for (int k = 0; k < COL_U; k++) v[k] = c + k < c1 ? cnt[(size_t)(c + k) * R + d] : 0u;
#pragma unroll
      for (int k = 0; k < COL_U; k++) t += v[k];
    }
    part[(size_t)b * R + d] = t;
  }
}

// One workgroup per (segment, 64 digits): lane = digit, wave g sums blocks
// g, g + G, ... of the segment (G waves).
template <int RB>
__global__ __launch_bounds__(1024) void coltot_kernel(const SortSeg* __restrict__ segs,
                                                      const uint64_t* __restrict__ part,
                                                      uint64_t* __restrict__ tot) {
  constexpr uint32_t R = 1u << RB;
  constexpr uint32_t DG = R / 64;               // digit groups per segment
  __shared__ uint64_t sm[16][64];
  const uint32_t s = blockIdx.x / DG, d = (blockIdx.x % DG) * 64 + __lane_id();
  const uint32_t G = blockDim.x >> 6, g = threadIdx.x >> 6;
  const SortSeg sg = segs[s];
  const uint32_t nb = (sg.chunk_end - sg.chunk_beg + COL_BLOCK_CHUNKS - 1) / COL_BLOCK_CHUNKS;
  uint64_t t = 0;
  for (uint32_t i = g; i < nb; i += G) t += part[(size_t)(sg.cblk_beg + i) * R + d];
  sm[g][__lane_id()] = t;
  __syncthreads();
  if (g == 0) {
    uint64_t all = 0;
    for (uint32_t q = 0; q < G; q++) all += sm[q][__lane_id()];
    tot[(size_t)s * R + d] = all;
  }
}

// One workgroup per (segment, 64 digits): lane = digit, wave g owns a
// contiguous run of the segment's blocks (G waves); the digit's base in the
// segment comes from the totals of the smaller digits.
template <int RB>
__global__ __launch_bounds__(1024) void colbase_kernel(const SortSeg* __restrict__ segs,
                                                       const uint64_t* __restrict__ tot,
                                                       uint64_t* __restrict__ part,
                                                       uint32_t* __restrict__ ticket) {
  constexpr uint32_t R = 1u << RB;
  constexpr uint32_t DG = R / 64;
  __shared__ uint64_t sm[16][64];
  __shared__ uint64_t s_below[16];
  // the scatter of this pass hands out its chunks from zero
  if (blockIdx.x == 0 && threadIdx.x == 0) *ticket = 0;
  const uint32_t s = blockIdx.x / DG, d0 = (blockIdx.x % DG) * 64;
  const uint32_t lane = __lane_id(), d = d0 + lane;
  const uint32_t G = blockDim.x >> 6, g = threadIdx.x >> 6;
  const SortSeg sg = segs[s];
  const uint64_t* tt = tot + (size_t)s * R;
  // records of the digits below this group's 64: every wave sums a share
  uint64_t below = 0;
  for (uint32_t q = threadIdx.x; q < d0; q += blockDim.x) below += tt[q];
  for (int o = 32; o > 0; o >>= 1) below += __shfl_xor(below, o);
  if (lane == 0) s_below[g] = below;
  // this wave's blocks: a contiguous run (a share of ceil(nb / G))
  const uint32_t nb = (sg.chunk_end - sg.chunk_beg + COL_BLOCK_CHUNKS - 1) / COL_BLOCK_CHUNKS;
  const uint32_t per = (nb + G - 1) / G;
  const uint32_t i0 = min(g * per, nb), i1 = min(i0 + per, nb);
  uint64_t* pd = part + (size_t)sg.cblk_beg * R + d;
  uint64_t mine = 0;
  for (uint32_t i = i0; i < i1; i++) mine += pd[(size_t)i * R];
  sm[g][lane] = mine;
  __syncthreads();
  uint64_t base = sg.beg;
  for (uint32_t q = 0; q < G; q++) base += s_below[q];
  // smaller digits of the group (an exclusive scan over the lanes)
  const uint64_t td = tt[d];
  uint64_t inc = td;
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t y = __shfl_up(inc, o);
    if (lane >= (uint32_t)o) inc += y;
  }
  base += inc - td;
  for (uint32_t q = 0; q < g; q++) base += sm[q][lane];   // earlier waves' blocks
  for (uint32_t i = i0; i < i1; i++) {
    const uint64_t v = pd[(size_t)i * R];
    pd[(size_t)i * R] = base;
    base += v;
  }
}

// Segments of few column blocks (at most COL_SMALL): totals, digit bases
// and block bases of a whole segment in one workgroup (one launch instead of
// the two above, whose cost on small logs is mostly the launch).
constexpr uint32_t COL_SMALL = 32;

template <int RB>
__global__ __launch_bounds__(1024) void colbase_small_kernel(const SortSeg* __restrict__ segs,
                                                             uint64_t* __restrict__ part,
                                                             uint32_t* __restrict__ ticket) {
  constexpr uint32_t R = 1u << RB;
  constexpr uint32_t PER = (R + 1023) / 1024;   // consecutive digits per thread
  __shared__ uint64_t s_tot[R];
  __shared__ uint64_t s_w[16];
  if (blockIdx.x == 0 && threadIdx.x == 0) *ticket = 0;
  const SortSeg sg = segs[blockIdx.x];
  const uint32_t nb = (sg.chunk_end - sg.chunk_beg + COL_BLOCK_CHUNKS - 1) / COL_BLOCK_CHUNKS;
  uint64_t* pb = part + (size_t)sg.cblk_beg * R;
  const uint32_t tid = threadIdx.x, lane = __lane_id(), w = tid >> 6;
  for (uint32_t d = tid; d < R; d += 1024) {
    uint64_t t = 0;
    for (uint32_t i = 0; i < nb; i++) t += pb[(size_t)i * R + d];
    s_tot[d] = t;
  }
  __syncthreads();
  // exclusive scan over the digits: thread tid owns digits [tid*PER, +PER)
  uint64_t mine = 0;
  for (uint32_t q = 0; q < PER; q++) {
    const uint32_t d = tid * PER + q;
    if (d < R) mine += s_tot[d];
  }
  uint64_t inc = mine;
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t y = __shfl_up(inc, o);
    if (lane >= (uint32_t)o) inc += y;
  }
  if (lane == 63) s_w[w] = inc;
  __syncthreads();
  uint64_t run = sg.beg + inc - mine;
  for (uint32_t v = 0; v < w; v++) run += s_w[v];
  __syncthreads();                      // every s_tot read above is done
  for (uint32_t q = 0; q < PER; q++) {
    const uint32_t d = tid * PER + q;
    if (d < R) {
      const uint64_t t = s_tot[d];
      s_tot[d] = run;                   // the digit's first slot in the segment
      run += t;
    }
  }
  __syncthreads();
  for (uint32_t d = tid; d < R; d += 1024) {
    uint64_t at = s_tot[d];
    for (uint32_t i = 0; i < nb; i++) {
      const uint64_t v = pb[(size_t)i * R + d];
      pb[(size_t)i * R + d] = at;
      at += v;
    }
  }
}

template <int RB>
__global__ __launch_bounds__(256) void coloff_kernel(const uint32_t* __restrict__ cnt,
                                                     const SortSeg* __restrict__ segs,
                                                     uint32_t nseg,
                                                     const uint64_t* __restrict__ part,
                                                     uint64_t* __restrict__ off) {
  constexpr uint32_t R = 1u << RB;
  const uint32_t b = blockIdx.x;
  const SortSeg sg = segs[cblk_seg(segs, nseg, b)];
  const uint32_t c0 = sg.chunk_beg + (b - sg.cblk_beg) * COL_BLOCK_CHUNKS;
  const uint32_t c1 = min(c0 + COL_BLOCK_CHUNKS, sg.chunk_end);
  for (uint32_t d = threadIdx.x; d < R; d += 256) {
    uint64_t at = part[(size_t)b * R + d];
    for (uint32_t c = c0; c < c1; c += COL_U) {
      uint32_t v[COL_U];
#pragma unroll
      for (int k = 0; k < COL_U; k++) v[k] = c + k < c1 ? cnt[(size_t)(c + k) * R + d] : 0u;
#pragma unroll
      for (int k = 0; k < COL_U; k++) {
        if (c + k < c1) off[(size_t)(c + k) * R + d] = at;
        at += v[k];
      }
    }
  }
}

// Stable scatter of one chunk, tile by tile (SC_BLOCK threads x SC_IPT
// records per tile).
// Ballot of v != 0 read straight from v (one compare; the compiler would
// otherwise rebuild the bit from the digit).
__device__ __forceinline__ uint64_t ballot_nonzero(uint32_t v) {
  uint64_t m;
  asm("v_cmp_ne_u32_e64 %0, 0, %1" : "=s"(m) : "v"(v));
  return m;
}

// Key loads of the scatter: plain, or streaming (non-temporal: the lines are
// not kept in the caches for reuse), which pays off on logs small enough for
// the caches to hold the output runs being written.
template <bool NTL>
__device__ __forceinline__ uint64_t load_key(const uint64_t* p) {
  if constexpr (NTL) return __builtin_nontemporal_load(p);
  else return *p;
}

template <int RB, int SC_BLOCK, int SC_IPT, bool NTL>
__global__ __launch_bounds__(SC_BLOCK) void scatter_kernel(const uint64_t* __restrict__ in,
                                                           uint64_t* __restrict__ out,
                                                           const SortChunk* __restrict__ chunks,
                                                           uint32_t nchunks,
                                                           const SortSeg* __restrict__ segs,
                                                           int lo, int nlo, int nbits,
                                                           const uint64_t* __restrict__ off,
                                                           uint32_t* __restrict__ ticket,
                                                           uint32_t* err,
                                                           void* __restrict__ dnext) {
  constexpr uint32_t R = 1u << RB;
  constexpr int SC_WAVES = SC_BLOCK / 64;
  constexpr uint32_t SC_TILE = SC_BLOCK * SC_IPT;
  __shared__ uint64_t sk[SC_TILE];              // the tile (in digit order after ranking)
  // per-wave digit counters (32-bit for the LDS adds of the ranking below
  // when they fit beside the tile, else 16-bit and updated item by item)
  constexpr bool RANK_ADD = SC_WAVES * R * 4 <= 32768;
  using HistT = typename std::conditional<RANK_ADD, uint32_t, uint16_t>::type;
  __shared__ HistT whist[SC_WAVES][R];         // per-wave counts, then prefixes
  __shared__ uint32_t lstart[R];               // tile-local digit starts
  __shared__ uint64_t grun[R];                 // next output slot per digit
  __shared__ uint64_t gofs[R];                 // grun - lstart for the tile
  __shared__ uint32_t scan_sm[SC_WAVES];
  __shared__ uint32_t s_next[2];               // chunk tickets, one chunk ahead

  const int tid = threadIdx.x, lane = __lane_id(), w = tid >> 6;
  const uint64_t lt = lanemask_lt();
  const uint32_t wbase = (uint32_t)w * 64 * SC_IPT;
  // persistent: workgroup b starts with chunk b and then takes chunk
  // gridDim.x + t for each ticket t it draws.  Thread 0 draws the ticket of
  // the chunk after next while the first tile of a chunk is ranked (slot
  // par of s_next; the next chunk's ticket is in slot par ^ 1), so the keys
  // of the next tile can be loaded, across chunk ends too, while the current
  // one is ranked and written.  A workgroup's tickets increase, so it stops
  // at its first ticket past the last chunk and drops no chunk.
  uint32_t ci = blockIdx.x;
  if (ci >= nchunks) return;
  if (tid == 0) s_next[1] = gridDim.x + atomicAdd(ticket, 1u);
  uint32_t par = 0;
  bool first_tile = true;
  SortChunk ch = chunks[ci];
  SortSeg sg = segs[ch.seg];
  // this pass's digit: key bits [lo, lo + RB); the next pass's, stored in
  // dnext as 1 byte (up to 8 bits) or 2: bits [nlo, nlo + nbits)
  int shift = (int)sg.shift + lo;
  int nshift = (int)sg.shift + nlo;
  const uint32_t nmask = (1u << nbits) - 1u;
  uint8_t* __restrict__ dn8 = nbits <= 8 ? static_cast<uint8_t*>(dnext) : nullptr;
  uint16_t* __restrict__ dn16 = nbits > 8 ? static_cast<uint16_t*>(dnext) : nullptr;
  for (uint32_t d = tid; d < R; d += SC_BLOCK) grun[d] = off[(size_t)ci * R + d];
  uint64_t base = ch.beg;
  // wave w owns records [w*64*IPT, (w+1)*64*IPT) of the tile; item k of
  // lane l is record w*64*IPT + k*64 + l (coalesced; rank order = input order)
  for (uint32_t q = tid; q < SC_WAVES * R; q += SC_BLOCK) (&whist[0][0])[q] = 0;
  __syncthreads();
  // Key loads are never conditional: a slot past the tile reads the tile's
  // last record (a tile is never empty), whose value goes unused.  A load
  // under a lane mask would sit behind a branch, and the wait for the
  // current tile's keys would then also wait for the next tile's loads.
  uint64_t key[SC_IPT];
  {
    const uint64_t rem = ch.end - base;
    const uint32_t n0 = rem < SC_TILE ? (uint32_t)rem : SC_TILE;
#pragma unroll
    for (int k = 0; k < SC_IPT; k++) {
      const uint32_t idx = wbase + k * 64 + lane;
      key[k] = load_key<NTL>(&in[base + (idx < n0 ? idx : n0 - 1)]);
    }
  }
  for (;;) {
    const uint64_t rem = ch.end - base;
    const uint32_t n_here = rem < SC_TILE ? (uint32_t)rem : SC_TILE;
    // the next tile: later in this chunk, else the first of the next chunk
    uint32_t nci = ci;
    uint64_t nbase = base + SC_TILE;
    SortChunk nch = ch;
    if (nbase >= ch.end) {
      nci = s_next[par ^ 1];
      if (nci < nchunks) {
        nch = chunks[nci];
        nbase = nch.beg;
      }
    }
    const bool has_next = nci < nchunks;
    uint64_t knext[SC_IPT];
    {
      // (no next tile: the current tile's first record, unused)
      const uint64_t nb = has_next ? nbase : base;
      const uint64_t nrem = has_next ? nch.end - nbase : 1;
      const uint32_t nn = nrem < SC_TILE ? (uint32_t)nrem : SC_TILE;
#pragma unroll
      for (int k = 0; k < SC_IPT; k++) {
        const uint32_t idx = wbase + k * 64 + lane;
        knext[k] = load_key<NTL>(&in[nb + (idx < nn ? idx : nn - 1)]);
      }
    }
    // Rank of each record among the wave's records of its digit, in input
    // order.  Per item: the lanes with the same digit (peers) from one ballot
    // per digit bit; the first peer adds the group's size to the wave's
    // counter of that digit and gets the count before it.  The adds of all
    // items are issued before any result is used (LDS serves one wave's
    // operations in order), then each group's base is fetched from its
    // first lane.
    uint32_t rank[SC_IPT], gbase[SC_IPT], first[SC_IPT];
#pragma unroll
    for (int k = 0; k < SC_IPT; k++) {
      const bool valid = (wbase + k * 64 + lane) < n_here;
      const uint32_t d = digit_at(key[k], shift, R - 1);
      const uint64_t act = __ballot(valid);
      uint64_t peers = act;
      // every active lane on one digit (long digit runs): no bit matching;
      // the valid lanes are a prefix of the wave, so lane 0 holds the first
      const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
      if (__ballot(valid && d == d0) != act) {
        // lanes whose digit differs from this lane's in some bit: for each
        // bit, its ballot XOR this lane's bit spread over 32 bits
        uint32_t diff_lo = 0, diff_hi = 0;
#pragma unroll
        for (int b = 0; b < RB; b++) {
          const uint32_t rep = (uint32_t)__builtin_amdgcn_sbfe((int)d, b, 1);   // 0 or ~0
          const uint64_t bb = ballot_nonzero(rep);
          diff_lo = __builtin_amdgcn_bitop3_b32(diff_lo, (uint32_t)bb, rep, 0xF6);   // a | (b ^ c)
          diff_hi = __builtin_amdgcn_bitop3_b32(diff_hi, (uint32_t)(bb >> 32), rep, 0xF6);
        }
        peers &= ~(((uint64_t)diff_hi << 32) | diff_lo);
      }
      const uint64_t below = peers & lt;
      rank[k] = (uint32_t)__popcll(below);
      if constexpr (RANK_ADD) {
        first[k] = (uint32_t)__builtin_ctzll(peers | (1ull << 63));   // lowest peer (63 if none)
        gbase[k] = 0;
        if (valid && below == 0) gbase[k] = atomicAdd(&whist[w][d], (uint32_t)__popcll(peers));
      } else {
        uint32_t before = 0;
        if (valid) before = whist[w][d];
        rank[k] += before;
        if (valid && below == 0) whist[w][d] = (HistT)(before + __popcll(peers));
        // lanes of a wave run in lock step; keep the next read after this write
        __builtin_amdgcn_wave_barrier();
      }
    }
    if constexpr (RANK_ADD) {
#pragma unroll
      for (int k = 0; k < SC_IPT; k++) rank[k] += __shfl(gbase[k], (int)first[k]);
    }
    if (first_tile && tid == 0) s_next[par] = gridDim.x + atomicAdd(ticket, 1u);
    first_tile = false;
    __syncthreads();
    {  // per digit: the waves' counts become prefixes over the waves; then
       // the tile-local exclusive scan over digits gives each digit's start
       // in the tile and its output offset, and the digit's next output slot
       // moves past this tile
      constexpr uint32_t PER = (R + SC_BLOCK - 1) / SC_BLOCK;
      uint32_t c[PER];
      uint32_t local = 0;
      for (uint32_t q = 0; q < PER; q++) {
        const uint32_t d = tid * PER + q;
        uint32_t run = 0;
        if (d < R) {
          for (int v = 0; v < SC_WAVES; v++) {
            const uint32_t x = whist[v][d];
            whist[v][d] = (HistT)run;
            run += x;
          }
        }
        c[q] = run;
        local += run;
      }
      uint32_t inc = local;
      for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
      }
      if (lane == 63) scan_sm[w] = inc;
      __syncthreads();
      uint32_t pre = 0;
      for (int v = 0; v < w; v++) pre += scan_sm[v];
      uint32_t run = pre + inc - local;
      for (uint32_t q = 0; q < PER; q++) {
        const uint32_t d = tid * PER + q;
        if (d < R) {
          lstart[d] = run;
          gofs[d] = grun[d] - run;
          grun[d] += c[q];
        }
        run += c[q];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SC_IPT; k++) {
      const bool valid = (wbase + k * 64 + lane) < n_here;
      if (valid) {
        const uint32_t d = digit_at(key[k], shift, R - 1);
        sk[lstart[d] + whist[w][d] + rank[k]] = key[k];
      }
    }
    __syncthreads();
    // digit runs out to the output (and each record's digit of the next
    // pass, which the next count pass reads, to dnext).  A destination
    // outside the segment can only come from inconsistent counts: it is
    // reported instead of written.  A full tile issues all its LDS reads
    // before any store.
    bool bad = false;
    const uint64_t seg_len = sg.end - sg.beg;
    if (n_here == SC_TILE) {
      // four records per thread at a time (registers stay few enough for
      // the occupancy the LDS allows)
      static_assert(SC_IPT % 4 == 0, "write-out in groups of four");
#pragma unroll 1
      for (int h = 0; h < SC_IPT; h += 4) {
        uint64_t kv[4], go[4];
#pragma unroll
        for (int k = 0; k < 4; k++) kv[k] = sk[tid + (h + k) * SC_BLOCK];
#pragma unroll
        for (int k = 0; k < 4; k++) go[k] = gofs[digit_at(kv[k], shift, R - 1)];
#pragma unroll
        for (int k = 0; k < 4; k++) {
          const uint64_t dst = go[k] + (uint32_t)(tid + (h + k) * SC_BLOCK);
          if (dst - sg.beg < seg_len) {
            out[dst] = kv[k];
            if (dn8) dn8[dst] = (uint8_t)digit_at(kv[k], nshift, nmask);
            else if (dn16) dn16[dst] = (uint16_t)digit_at(kv[k], nshift, nmask);
          } else {
            bad = true;
          }
        }
      }
    } else {
      for (uint32_t p = tid; p < n_here; p += SC_BLOCK) {
        const uint64_t kv = sk[p];
        const uint64_t dst = gofs[digit_at(kv, shift, R - 1)] + p;
        if (dst - sg.beg < seg_len) {
          out[dst] = kv;
          if (dn8) dn8[dst] = (uint8_t)digit_at(kv, nshift, nmask);
          else if (dn16) dn16[dst] = (uint16_t)digit_at(kv, nshift, nmask);
        } else {
          bad = true;
        }
      }
    }
    if (bad) atomicOr(err, ERR_RANGE);
    // the wave counters are free again: clear them for the next tile
    for (uint32_t q = tid; q < SC_WAVES * R; q += SC_BLOCK) (&whist[0][0])[q] = 0;
    __syncthreads();
    if (!has_next) break;
    if (nci != ci) {
      ci = nci;
      par ^= 1;
      first_tile = true;
      ch = nch;
      sg = segs[ch.seg];
      shift = (int)sg.shift + lo;
      nshift = (int)sg.shift + nlo;
      for (uint32_t d = tid; d < R; d += SC_BLOCK) grun[d] = off[(size_t)ci * R + d];
    }
    base = nbase;
#pragma unroll
    for (int k = 0; k < SC_IPT; k++) key[k] = knext[k];
  }
}

uint32_t sort_tile_size() { return SC_MAX_TILE; }

#define RB_SWITCH(rb, CALL)                             \
  switch (rb) {                                         \
    case 6: { constexpr int RBV = 6; CALL; } break;     \
    case 7: { constexpr int RBV = 7; CALL; } break;     \
    case 8: { constexpr int RBV = 8; CALL; } break;     \
    case 9: { constexpr int RBV = 9; CALL; } break;     \
    case 10: { constexpr int RBV = 10; CALL; } break;   \
    case 11: { constexpr int RBV = 11; CALL; } break;   \
    default: return hipErrorInvalidValue;               \
  }

hipError_t launch_sort_scan(int rb, const void* dig, const SortSeg* segs, uint32_t nseg,
                            const SortChunk* chunks, uint32_t nchunks, uint32_t n_cblk,
                            uint32_t max_cblk, uint32_t* cnt, uint64_t* tot, uint64_t* part,
                            uint64_t* off, uint32_t* ticket, bool counts_ready, hipStream_t s) {
  if (nchunks == 0) return hipSuccess;
  const uint32_t R = 1u << rb;
  if (!counts_ready) {
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    const uint32_t grid = std::min<uint32_t>(nchunks, (uint32_t)ncu * 8);
    RB_SWITCH(rb, (count_kernel<RBV><<<grid, 64 * CNT_WAVES, 0, s>>>((const DigT<RBV>*)dig, chunks,
                                                                     nchunks, cnt)));
  }
  // waves per (segment, 64 digits) workgroup: enough that each walks a few
  // column blocks of the longest segment, at most 16
  uint32_t G = 1;
  while (G < 16 && G * 4 < max_cblk) G <<= 1;
  const uint32_t dgrid = nseg * (R / 64);
  RB_SWITCH(rb, (colpart_kernel<RBV><<<n_cblk, 256, 0, s>>>(cnt, segs, nseg, part)));
  if (max_cblk <= COL_SMALL) {
    RB_SWITCH(rb, (colbase_small_kernel<RBV><<<nseg, 1024, 0, s>>>(segs, part, ticket)));
  } else {
    RB_SWITCH(rb, (coltot_kernel<RBV><<<dgrid, 64 * G, 0, s>>>(segs, part, tot)));
    RB_SWITCH(rb, (colbase_kernel<RBV><<<dgrid, 64 * G, 0, s>>>(segs, tot, part, ticket)));
  }
  RB_SWITCH(rb, (coloff_kernel<RBV><<<n_cblk, 256, 0, s>>>(cnt, segs, nseg, part, off)));
  return hipGetLastError();
}

static int g_scatter_variant = 4;   // 512 threads x 8 records: best measured default
int scatter_variant(int v, bool set) {
  const int old = g_scatter_variant;
  if (set) g_scatter_variant = v;
  return old;
}
// per-pass shapes: 4 bits per pass in execution order (passes 0..6), 15 =
// the shape above
static int g_pass_shapes = PASS_SHAPES_DEFAULT;
int pass_shapes(int v, bool set) {
  const int old = g_pass_shapes;
  if (set) g_pass_shapes = v;
  return old;
}
static int g_scatter_wgs = 0;       // workgroups per CU; 0 = the occupancy query's answer
int scatter_wgs(int v, bool set) {
  const int old = g_scatter_wgs;
  if (set) g_scatter_wgs = v;
  return old;
}

template <int RB, int BLOCK, int IPT, bool NTL = false>
static void scatter_go(uint32_t nchunks, const uint64_t* in, uint64_t* out,
                       const SortChunk* chunks, const SortSeg* segs, int lo, int nlo, int nbits,
                       const uint64_t* off, uint32_t* ticket, uint32_t* err, void* dnext,
                       hipStream_t s) {
  int dev = 0, ncu = 256, per_cu = 0;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (g_scatter_wgs > 0)
    per_cu = g_scatter_wgs;
  else if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, scatter_kernel<RB, BLOCK, IPT, NTL>,
                                                         BLOCK, 0) != hipSuccess ||
           per_cu < 1)
    per_cu = 1;
  uint32_t grid = (uint32_t)ncu * (uint32_t)per_cu;
  if (grid > nchunks) grid = nchunks;
  scatter_kernel<RB, BLOCK, IPT, NTL><<<grid, BLOCK, 0, s>>>(in, out, chunks, nchunks, segs, lo, nlo, nbits, off, ticket,
                                                              err, dnext);
}

template <int RB>
static void scatter_launch(int variant, uint32_t nchunks, const uint64_t* in, uint64_t* out,
                           const SortChunk* chunks, const SortSeg* segs, int lo, int nlo, int nbits,
                           const uint64_t* off, uint32_t* ticket, uint32_t* err, void* dn,
                           hipStream_t s) {
  switch (variant) {
    case 1: scatter_go<RB, 256, 16>(nchunks, in, out, chunks, segs, lo, nlo, nbits, off, ticket, err, dn, s); break;
    case 2: scatter_go<RB, 256, 32>(nchunks, in, out, chunks, segs, lo, nlo, nbits, off, ticket, err, dn, s); break;
    case 4: scatter_go<RB, 512, 8>(nchunks, in, out, chunks, segs, lo, nlo, nbits, off, ticket, err, dn, s); break;
    case 5: scatter_go<RB, 1024, 4>(nchunks, in, out, chunks, segs, lo, nlo, nbits, off, ticket, err, dn, s); break;
    case 6: scatter_go<RB, 256, 8>(nchunks, in, out, chunks, segs, lo, nlo, nbits, off, ticket, err, dn, s); break;
    case 7:
      scatter_go<RB, 512, 8, true>(nchunks, in, out, chunks, segs, lo, nlo, nbits, off, ticket, err, dn, s);
      break;
    case 9:
      scatter_go<RB, 512, 16, true>(nchunks, in, out, chunks, segs, lo, nlo, nbits, off, ticket, err, dn, s);
      break;
    case 8:
      if constexpr (RB <= 9)
        scatter_go<RB, 1024, 8, true>(nchunks, in, out, chunks, segs, lo, nlo, nbits, off, ticket, err, dn, s);
      else
        scatter_go<RB, 512, 16, true>(nchunks, in, out, chunks, segs, lo, nlo, nbits, off, ticket, err, dn, s);
      break;
    case 3:
      // 16 waves of per-digit counters do not fit LDS beside the tile for
      // wide digits
      if constexpr (RB <= 9) {
        scatter_go<RB, 1024, 8>(nchunks, in, out, chunks, segs, lo, nlo, nbits, off, ticket, err, dn, s);
        break;
      }
      [[fallthrough]];
    default: scatter_go<RB, 512, 16>(nchunks, in, out, chunks, segs, lo, nlo, nbits, off, ticket, err, dn, s); break;
  }
}

hipError_t launch_sort_scatter(int rb, int pass, const uint64_t* in, uint64_t* out,
                               const SortSeg* segs, const SortChunk* chunks, uint32_t nchunks,
                               int lo, int nlo, int nbits, const uint64_t* off, uint32_t* ticket,
                               uint32_t* err, void* dnext, hipStream_t s) {
  if (nchunks == 0) return hipSuccess;
  const int own = pass < 7 ? (g_pass_shapes >> (4 * pass)) & 15 : 15;
  const int v = own <= SCATTER_SHAPE_MAX ? own : g_scatter_variant;
  RB_SWITCH(rb, (scatter_launch<RBV>(v, nchunks, in, out, chunks, segs, lo, nlo, nbits, off, ticket, err,
                                     dnext, s)));
  return hipGetLastError();
}

}  // namespace rp

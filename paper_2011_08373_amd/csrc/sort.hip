// Stable LSD radix sort of the access records, one launch per digit pass.
//
// Single-pass ("onesweep") scheme for CDNA4: each 512-thread workgroup takes
// the next tile of 8192 records (tile ids come from an atomic counter, so a
// tile only ever waits for tiles that already started), ranks the keys of
// its tile stably with 64-lane ballots, publishes its digit counts, obtains
// the records of earlier tiles with the same digit by decoupled look-back,
// stages the tile in LDS in digit order and writes digit runs out in order.
// Global digit offsets of every pass come from the histograms counted while
// the records were generated.  Several sort segments (logs) are sorted by
// one launch; look-back never crosses a segment's first tile.
//
// The look-back wait is bounded: a tile that waits too long records an error
// (checked by the host) and carries on, so the grid always drains.
#include "common.h"
#include "launch.h"

namespace rp {

constexpr int SORT_BLOCK = 512;
constexpr int SORT_WAVES = SORT_BLOCK / 64;
constexpr int SORT_IPT = 16;
constexpr uint32_t SORT_TILE = SORT_BLOCK * SORT_IPT;  // 8192 records
constexpr uint64_t FLAG_AGG = 1ull << 62, FLAG_INC = 2ull << 62;
constexpr uint64_t VAL_MASK = (1ull << 62) - 1;
constexpr uint32_t SPIN_LIMIT = 1u << 22;

__global__ void fill_u64_kernel(uint64_t* p, uint64_t n, uint64_t v) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

__device__ __forceinline__ void st_status(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_status(uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int RB>
__global__ __launch_bounds__(SORT_BLOCK) void onesweep_kernel(
    const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
    const SortSeg* __restrict__ segs, int nseg, int pass, int passes,
    const uint64_t* __restrict__ dbase, uint64_t* status, uint32_t* counter, uint32_t* err) {
  constexpr uint32_t R = 1u << RB;
  __shared__ uint64_t sk[SORT_TILE];                // 64 KiB
  __shared__ uint16_t whist[SORT_WAVES][R];         // per-wave counts, then prefixes
  __shared__ uint32_t lstart[R];                    // tile-local digit starts
  __shared__ uint64_t gexcl[R];                     // global offset of the tile's digit run
  __shared__ uint32_t s_tile, s_seg;
  __shared__ uint32_t scan_sm[SORT_WAVES];

  const int tid = threadIdx.x, lane = __lane_id(), w = tid >> 6;
  if (tid == 0) {
    const uint32_t t = atomicAdd(counter, 1u);
    int lo = 0, hi = nseg - 1;           // largest segment with tile_beg <= t
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (segs[mid].tile_beg <= t) lo = mid; else hi = mid - 1;
    }
    s_tile = t;
    s_seg = (uint32_t)lo;
  }
  for (uint32_t q = tid; q < SORT_WAVES * R; q += SORT_BLOCK) (&whist[0][0])[q] = 0;
  __syncthreads();
  const uint32_t tile = s_tile, segi = s_seg;
  const SortSeg sg = segs[segi];
  const uint32_t tin = tile - sg.tile_beg;
  const uint64_t base = sg.beg + (uint64_t)tin * SORT_TILE;
  const uint64_t rem = sg.end - base;
  const uint32_t n_here = rem < SORT_TILE ? (uint32_t)rem : SORT_TILE;
  const int shift = (int)sg.shift + pass * RB;

  // load: wave w owns 64*IPT consecutive records, item k of lane l is record
  // w*64*IPT + k*64 + l (coalesced; rank order == input order)
  uint64_t key[SORT_IPT];
  uint32_t rank[SORT_IPT];
  const uint32_t wbase = (uint32_t)w * 64 * SORT_IPT;
#pragma unroll
  for (int k = 0; k < SORT_IPT; k++) {
    const uint32_t idx = wbase + k * 64 + lane;
    key[k] = idx < n_here ? in[base + idx] : 0;
  }
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int k = 0; k < SORT_IPT; k++) {
    const bool valid = (wbase + k * 64 + lane) < n_here;
    const uint32_t d = digit_at(key[k], shift, R - 1);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < RB; b++) {
      const bool bit = (d >> b) & 1;
      const uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    uint32_t before = 0;
    if (valid) before = whist[w][d];
    rank[k] = before + (uint32_t)__popcll(peers & lt);
    if (valid && (peers & lt) == 0) whist[w][d] = (uint16_t)(before + __popcll(peers));
    // the wave's lanes run in lock step; keep the compiler from moving the
    // next item's counter read above this write
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();

  // per digit: prefix over waves, tile count, publish, look back
  for (uint32_t d = tid; d < R; d += SORT_BLOCK) {
    uint32_t run = 0;
    for (int v = 0; v < SORT_WAVES; v++) {
      const uint32_t c = whist[v][d];
      whist[v][d] = (uint16_t)run;
      run += c;
    }
    lstart[d] = run;  // tile count for now
    uint64_t* my = status + (uint64_t)tile * R + d;
    if (tin == 0) {
      const uint64_t g = dbase[((size_t)segi * passes + pass) * R + d];
      st_status(my, FLAG_INC | (g + run));
      gexcl[d] = g;
    } else {
      st_status(my, FLAG_AGG | run);
    }
  }
  for (uint32_t d = tid; d < R; d += SORT_BLOCK) {
    if (tin == 0) continue;
    uint64_t excl = 0;
    uint32_t t = tile - 1;
    uint32_t spins = 0;
    for (;;) {
      const uint64_t s = ld_status(status + (uint64_t)t * R + d);
      const uint64_t f = s & ~VAL_MASK;
      if (f == 0) {
        if (++spins > SPIN_LIMIT) { atomicOr(err, ERR_SORT); break; }
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      excl += s & VAL_MASK;
      if (f == FLAG_INC || t == sg.tile_beg) break;
      t--;
    }
    st_status(status + (uint64_t)tile * R + d, FLAG_INC | (excl + lstart[d]));
    gexcl[d] = excl;
  }
  __syncthreads();

  // tile-local exclusive scan of the digit counts -> lstart
  {
    constexpr uint32_t PER = (R + SORT_BLOCK - 1) / SORT_BLOCK;
    uint32_t c[PER];
    uint32_t local = 0;
    for (uint32_t q = 0; q < PER; q++) {
      const uint32_t d = tid * PER + q;
      c[q] = d < R ? lstart[d] : 0;
      local += c[q];
    }
    uint32_t inc = local;
    for (int off = 1; off < 64; off <<= 1) {
      uint32_t y = __shfl_up(inc, off);
      if (lane >= off) inc += y;
    }
    if (lane == 63) scan_sm[w] = inc;
    __syncthreads();
    uint32_t pre = 0;
    for (int v = 0; v < w; v++) pre += scan_sm[v];
    uint32_t run = pre + inc - local;
    __syncthreads();
    for (uint32_t q = 0; q < PER; q++) {
      const uint32_t d = tid * PER + q;
      if (d < R) lstart[d] = run;
      run += c[q];
    }
  }
  __syncthreads();

  // scatter into LDS in digit order
#pragma unroll
  for (int k = 0; k < SORT_IPT; k++) {
    const bool valid = (wbase + k * 64 + lane) < n_here;
    if (valid) {
      const uint32_t d = digit_at(key[k], shift, R - 1);
      sk[lstart[d] + whist[w][d] + rank[k]] = key[k];
    }
  }
  __syncthreads();
  // write digit runs in order (consecutive threads -> consecutive addresses)
  for (uint32_t p = tid; p < n_here; p += SORT_BLOCK) {
    const uint64_t kv = sk[p];
    const uint32_t d = digit_at(kv, shift, R - 1);
    const uint64_t dst = gexcl[d] + (p - lstart[d]);
    // a destination outside the segment can only come from inconsistent
    // counts: report it instead of writing
    if (dst >= sg.beg && dst < sg.end) out[dst] = kv;
    else atomicOr(err, ERR_RANGE);
  }
}

uint32_t sort_tile_size() { return SORT_TILE; }

hipError_t launch_fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  fill_u64_kernel<<<(uint32_t)blocks, 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_sort_pass(int rb, const uint64_t* in, uint64_t* out, const SortSeg* segs,
                            int nseg, uint32_t n_tiles, int pass, int passes,
                            const uint64_t* dbase, uint64_t* status, uint32_t* counter,
                            uint32_t* err, hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  switch (rb) {
    case 8: onesweep_kernel<8><<<n_tiles, SORT_BLOCK, 0, s>>>(in, out, segs, nseg, pass, passes, dbase, status, counter, err); break;
    case 9: onesweep_kernel<9><<<n_tiles, SORT_BLOCK, 0, s>>>(in, out, segs, nseg, pass, passes, dbase, status, counter, err); break;
    case 10: onesweep_kernel<10><<<n_tiles, SORT_BLOCK, 0, s>>>(in, out, segs, nseg, pass, passes, dbase, status, counter, err); break;
    case 11: onesweep_kernel<11><<<n_tiles, SORT_BLOCK, 0, s>>>(in, out, segs, nseg, pass, passes, dbase, status, counter, err); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace rp

// Access-record generation.
//
// One work item writes a contiguous run of records of one log: the
// same-block log in block-major order, the cross-block log (GLOBAL arrays
// only) in point-major order; common.h describes the packing.  Each record
// is a pure function of (point, block, thread): the word is
// (a*tid + b*bid + c) mod words (Euclidean residue), and the executing
// threads are those with tid % m == r of the blocks with bid % bm == br.
// The same-block log keeps the same number of records for every block: a
// block that does not execute a point gets padding records in its place,
// all in one location of their own (array id pad_array, word 0, that block)
// and all of thread 0, so they never conflict with anything.  The
// cross-block log holds the executing blocks only.  Items coincide with the sort's
// chunks: while writing, an item counts the radix digits of the first sort
// pass in LDS and stores them as its chunk's count row.  The item's points
// (up to 256, from its first point on, which the host finds) are staged in
// LDS first.
#include "common.h"
#include "launch.h"

namespace rp {

constexpr int GEN_BLOCK = 256;
constexpr uint32_t GEN_CACHE = 256;   // points staged in LDS per item

// Counts the digit of each valid lane's record (the valid lanes are a
// prefix of the wave): one LDS add for the whole wave when every valid lane
// has lane 0's digit (the usual case for the key's top digit, which the
// records of one point and block mostly share; 64 adds to one counter
// would be served one after another), else one add per record (no return
// value, so the adds do not stall the wave).
template <int RB>
__device__ __forceinline__ void count_digits(uint32_t* hist, uint64_t rec, int shift, bool valid) {
  constexpr uint32_t R = 1u << RB;
  const uint32_t d = digit_at(rec, shift, R - 1);
  const uint64_t act = __builtin_amdgcn_ballot_w64(valid);
  const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
  if ((__builtin_amdgcn_ballot_w64(d == d0) & act) == act) {
    if (__lane_id() == 0 && act) atomicAdd(&hist[d0], (uint32_t)__popcll(act));
  } else if (valid) {
    atomicAdd(&hist[d], 1u);
  }
}

// Digit counts of a wave's steps.  A step whose valid lanes all carry one
// digit adds its count to a wave-uniform run (scalar registers), which is
// added to the LDS counter with one add when the digit changes or the wave
// is done; other steps add each record on its own.  The valid lanes are a
// prefix of the wave (lane 0 is always one of them).
struct DigitRun {
  uint32_t d = 0, n = 0;
  __device__ __forceinline__ void flush(uint32_t* hist) {
    if (n != 0 && __lane_id() == 0) atomicAdd(&hist[d], n);
    n = 0;
  }
  __device__ __forceinline__ void add(uint32_t* hist, uint32_t dd, uint32_t k) {
    if (dd != d) {
      flush(hist);
      d = dd;
    }
    n += k;
  }
};
template <int RB>
__device__ __forceinline__ void count_step(uint32_t* hist, DigitRun& run, uint64_t rec, int shift,
                                           bool valid, uint64_t act) {
  constexpr uint32_t R = 1u << RB;
  const uint32_t d = digit_at(rec, shift, R - 1);
  const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
  if (act == 0) return;                     // a wave wholly past the end
  if ((__builtin_amdgcn_ballot_w64(d == d0) & act) == act)
    run.add(hist, d0, (uint32_t)__popcll(act));
  else if (valid)
    atomicAdd(&hist[d], 1u);
}

// Wave-uniform copies (the values are the same in every lane; saying so
// keeps the per-point arithmetic on the scalar unit).
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
  return ((uint64_t)uni((uint32_t)(v >> 32)) << 32) | uni((uint32_t)v);
}
__device__ __forceinline__ DPoint uni_point(const DPoint& p) {
  static_assert(sizeof(DPoint) == 40, "ten words");
  DPoint u;
  const uint32_t* s = reinterpret_cast<const uint32_t*>(&p);
  uint32_t* d = reinterpret_cast<uint32_t*>(&u);
#pragma unroll
  for (int k = 0; k < 10; k++) d[k] = uni(s[k]);
  return u;
}
// x * tid for a wave-uniform x: one 24-bit multiply when x fits (the usual
// case: strides and guard moduli are small), else a full one; the product is
// taken mod 2^32 either way.
__device__ __forceinline__ uint32_t mul_tid(uint32_t x, uint32_t tid) {
  const int32_t xs = (int32_t)x;
  if (xs >= -(1 << 23) && xs < (1 << 23)) return (uint32_t)__mul24(xs, (int32_t)tid);
  return x * tid;
}

template <int RB>
__global__ __launch_bounds__(GEN_BLOCK) void gen_kernel(const GenItem* __restrict__ items,
                                                        const Job* __restrict__ jobs,
                                                        const SortSeg* __restrict__ segs,
                                                        uint64_t* __restrict__ recs,
                                                        uint32_t* __restrict__ item_hist,
                                                        int count_lo) {
  constexpr uint32_t R = 1u << RB;
  __shared__ uint32_t hist[R];
  __shared__ DPoint s_pts[GEN_CACHE];        // points i0, i0+1, ... (mod P) of the item
  __shared__ uint64_t s_cnt[GEN_CACHE];      // their records (per block in the same-block log)
  __shared__ uint64_t s_pre[GEN_CACHE];      // their prefix entries
  const GenItem it = items[blockIdx.x];
  const Job& J = jobs[it.job];
  const SortSeg sg = segs[it.seg];
  const int count = count_lo >= 0;
  const int shift = (int)sg.shift + (count ? count_lo : 0);
  const uint32_t tid = threadIdx.x;
  uint64_t* out = recs + sg.beg;
  for (uint32_t q = tid; q < R; q += GEN_BLOCK) hist[q] = 0;
  const uint32_t ks = J.key_shift, tb = J.tbits, bb = J.bbits, pb = J.pbits, nb = J.nbits;
  const uint32_t P = J.P;
  const uint64_t* pre = it.view == 0 ? J.cnt_pre : J.gcnt_pre;
  const uint64_t first = it.view == 0 ? it.o0 % J.rblk : it.o0;
  const uint32_t i0 = it.i0;                 // point holding record o0 (set by the host)
  const uint32_t nc = P < GEN_CACHE ? P : GEN_CACHE;
  for (uint32_t d = tid; d < nc; d += GEN_BLOCK) {
    uint32_t i = i0 + d;
    if (i >= P) i -= P;
    s_pts[d] = J.pts[i];
    s_pre[d] = pre[i];
    s_cnt[d] = pre[i + 1] - pre[i];
  }
  __syncthreads();
  if (it.view == 0) {
    // block-major: block k, points in order, executing threads in order.
    // Segment s of the item is point (i0 + s) mod P of block k0 + (i0 + s) / P;
    // its records are a contiguous stretch, and wave w takes segments w,
    // w + WAVES, ... (a segment usually has a few hundred records, so one wave
    // covers it in a few steps and the per-segment work is paid once per wave)
    constexpr uint32_t WAVES = GEN_BLOCK / 64;
    const uint32_t w = uni(tid >> 6), lane = tid & 63u;
    const uint64_t rblk = J.rblk;
    uint32_t k = (uint32_t)(it.o0 / rblk);
    DigitRun run;
    uint32_t sd = w;                   // segment index (cache slot while < nc)
    uint32_t si = i0 + w;
    while (si >= P) { si -= P; k++; }
    for (;;) {
      const bool cached = sd < nc;
      const uint64_t pbeg = uni64(cached ? s_pre[sd] : pre[si]);
      const uint64_t sbeg = (uint64_t)k * rblk + pbeg;     // first record of the segment
      if (sbeg >= it.o1) break;
      const uint64_t c = uni64(cached ? s_cnt[sd] : pre[si + 1] - pre[si]);
      const uint64_t lo = sbeg > it.o0 ? sbeg : it.o0;
      const uint64_t hi = sbeg + c < it.o1 ? sbeg + c : it.o1;
      if (lo < hi) {
        const DPoint p = uni_point(cached ? s_pts[sd] : J.pts[si]);
        const uint64_t low = ((uint64_t)k << (pb + tb)) | ((uint64_t)si << tb);
        // (a segment is one point of one block: fewer than 2^32 records)
        const uint32_t take = uni((uint32_t)(hi - lo));
        const uint32_t nfull = take >> 6, rem = take & 63u;
        uint64_t* const dst = out + lo;
        if (p.bm > 1 && k % p.bm != p.br) {
          // this block does not execute the point: padding, one record for
          // the whole segment
          const uint64_t rec = (((uint64_t)J.pad_array << nb) << ks) | low;
          for (uint32_t st = 0; st < nfull; st++) dst[st * 64 + lane] = rec;
          if (lane < rem) dst[nfull * 64 + lane] = rec;
          if (count) run.add(hist, uni(digit_at(rec, shift, R - 1)), take);
        } else {
          const uint64_t arr = (uint64_t)p.array << nb;
          // record u0 + q of the point: thread t = r + m*(u0 + q)
          const uint32_t u0 = (uint32_t)(lo - sbeg);
          const uint32_t t0 = p.r + p.m * u0;
          const uint32_t mt = mul_tid(p.m, lane);
          // power-of-two words: word = (a*t + b*k + c) mod 2^32, masked
          const bool pow2 = p.flags & PF_POW2;
          const uint32_t am = (uint32_t)p.a * p.m;
          const uint32_t at = pow2 ? mul_tid(am, lane) : 0u;
          const uint32_t cw = (uint32_t)p.a * t0 + (uint32_t)p.b * k + (uint32_t)p.c;
          const uint32_t wmask = p.words - 1;
          auto record = [&](uint32_t q0) {
            const uint32_t t = t0 + p.m * q0 + mt;
            const uint32_t word = pow2 ? (cw + am * q0 + at) & wmask : word_of(p, t, k);
            return ((arr | word) << ks) | low | t;
          };
          // whole steps with no lane mask, then the tail
          for (uint32_t st = 0; st < nfull; st++) {
            const uint64_t rec = record(st * 64);
            dst[st * 64 + lane] = rec;
            if (count) count_step<RB>(hist, run, rec, shift, true, ~0ull);
          }
          if (rem) {
            const bool valid = lane < rem;
            const uint64_t rec = record(nfull * 64);
            if (valid) dst[nfull * 64 + lane] = rec;
            if (count) count_step<RB>(hist, run, rec, shift, valid, __ballot(valid));
          }
        }
      }
      sd += WAVES;
      si += WAVES;
      while (si >= P) { si -= P; k++; }
    }
    if (count) run.flush(hist);
  } else {
    // point-major over GLOBAL access points: point i, executing blocks in
    // order, executing threads in order (one thread when the word does not
    // depend on it; the first two executing blocks only when it does not
    // depend on the block)
    DigitRun run;
    uint32_t i = i0;
    uint32_t d = 0;            // cache slot of point i
    uint64_t pos = it.o0;
    uint64_t j0 = first - pre[i];
    while (pos < it.o1) {
      const bool cached = d < nc;
      const uint64_t span = uni64(cached ? s_cnt[d] : pre[i + 1] - pre[i]);
      const uint64_t take = (span - j0) < (it.o1 - pos) ? (span - j0) : (it.o1 - pos);
      if (take) {
        const DPoint p = uni_point(cached ? s_pts[d] : J.pts[i]);
        const uint32_t cnt = (p.flags & PF_TCONST) ? 1u : p.cnt;
        const uint64_t arr = (uint64_t)p.array << nb;
        const uint64_t pf = (uint64_t)i << (bb + tb);
        // record j of the point: block j / cnt, its (j mod cnt)-th executing thread
        const bool cpow2 = (cnt & (cnt - 1)) == 0;
        const uint32_t csh = 31u - (uint32_t)__builtin_clz(cnt);
        const bool pow2 = p.flags & PF_POW2;
        const uint32_t wmask = p.words - 1;
        auto record = [&](uint64_t q) {
          const uint64_t j = j0 + q;
          uint32_t kk, u;
          if (cpow2 && span < (1ull << 32)) {
            kk = (uint32_t)j >> csh;
            u = (uint32_t)j & (cnt - 1);
          } else if (span < (1ull << 32)) {
            kk = (uint32_t)j / cnt;
            u = (uint32_t)j - kk * cnt;
          } else {
            kk = (uint32_t)(j / cnt);
            u = (uint32_t)(j - (uint64_t)kk * cnt);
          }
          const uint32_t t = p.r + p.m * u;
          kk = p.br + p.bm * kk;           // the kk-th executing block
          uint32_t word;
          if (pow2) word = ((uint32_t)p.a * t + (uint32_t)p.b * kk + (uint32_t)p.c) & wmask;
          else word = word_of(p, t, kk);
          return ((arr | word) << ks) | pf | ((uint64_t)kk << tb);
        };
        // whole steps of the workgroup with no lane mask, then the tail
        const uint64_t nfull = uni64(take / GEN_BLOCK);
        uint64_t* const dst = out + pos;
        for (uint64_t st = 0; st < nfull; st++) {
          const uint64_t q = st * GEN_BLOCK + tid;
          const uint64_t rec = record(q);
          dst[q] = rec;
          if (count) count_step<RB>(hist, run, rec, shift, true, ~0ull);
        }
        if (nfull * GEN_BLOCK < take) {
          const uint64_t q = nfull * GEN_BLOCK + tid;
          const bool valid = q < take;
          const uint64_t rec = record(q);
          if (valid) dst[q] = rec;
          if (count) count_step<RB>(hist, run, rec, shift, valid, __ballot(valid));
        }
      }
      pos += take;
      j0 = 0;
      d++;
      i++;
    }
    if (count) run.flush(hist);
  }
  if (!count) return;
  __syncthreads();
  uint32_t* row = item_hist + (size_t)blockIdx.x * R;
  for (uint32_t q = tid; q < R; q += GEN_BLOCK) row[q] = hist[q];
}

// One thread per chunk: its segment (the last with chunk_beg <= c), its
// record range and the point holding its first record (the last i with
// pre[i] <= offset, the offset taken within one block for the same-block
// log).
__global__ __launch_bounds__(256) void items_kernel(const Job* __restrict__ jobs,
                                                    const SortSeg* __restrict__ segs, uint32_t nseg,
                                                    uint32_t nchunks, uint64_t chunk_len,
                                                    GenItem* __restrict__ items,
                                                    SortChunk* __restrict__ chunks) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nchunks) return;
  uint32_t lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (segs[mid].chunk_beg <= c) lo = mid; else hi = mid - 1;
  }
  const SortSeg sg = segs[lo];
  const uint64_t n = sg.end - sg.beg;
  const uint64_t o0 = (uint64_t)(c - sg.chunk_beg) * chunk_len;
  const uint64_t o1 = o0 + chunk_len < n ? o0 + chunk_len : n;
  const Job& J = jobs[sg.job];
  const uint64_t* pre = sg.view == 0 ? J.cnt_pre : J.gcnt_pre;
  const uint64_t first = sg.view == 0 ? o0 % J.rblk : o0;
  uint32_t a = 0, b = J.P;            // the first i in [0, P) with pre[i] > first, or P
  while (a < b) {
    const uint32_t mid = (a + b) >> 1;
    if (pre[mid] <= first) a = mid + 1; else b = mid;
  }
  GenItem it;
  it.o0 = o0;
  it.o1 = o1;
  it.job = sg.job;
  it.view = sg.view;
  it.seg = lo;
  it.i0 = a - 1;
  items[c] = it;
  SortChunk ch;
  ch.beg = sg.beg + o0;
  ch.end = sg.beg + o1;
  ch.seg = lo;
  ch.pad = 0;
  chunks[c] = ch;
}

hipError_t launch_items(const Job* jobs, const SortSeg* segs, uint32_t nseg, uint32_t nchunks,
                        uint64_t chunk_len, GenItem* items, SortChunk* chunks, hipStream_t s) {
  if (nchunks == 0 || nseg == 0) return hipSuccess;
  items_kernel<<<(nchunks + 255) / 256, 256, 0, s>>>(jobs, segs, nseg, nchunks, chunk_len, items,
                                                     chunks);
  return hipGetLastError();
}

hipError_t launch_gen(int rb, const GenItem* items, uint32_t n_items, const Job* jobs,
                      const SortSeg* segs, uint64_t* recs, uint32_t* item_hist, int count_lo,
                      hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  switch (rb) {
    case 6: gen_kernel<6><<<n_items, GEN_BLOCK, 0, s>>>(items, jobs, segs, recs, item_hist, count_lo); break;
    case 7: gen_kernel<7><<<n_items, GEN_BLOCK, 0, s>>>(items, jobs, segs, recs, item_hist, count_lo); break;
    case 8: gen_kernel<8><<<n_items, GEN_BLOCK, 0, s>>>(items, jobs, segs, recs, item_hist, count_lo); break;
    case 9: gen_kernel<9><<<n_items, GEN_BLOCK, 0, s>>>(items, jobs, segs, recs, item_hist, count_lo); break;
    case 10: gen_kernel<10><<<n_items, GEN_BLOCK, 0, s>>>(items, jobs, segs, recs, item_hist, count_lo); break;
    case 11: gen_kernel<11><<<n_items, GEN_BLOCK, 0, s>>>(items, jobs, segs, recs, item_hist, count_lo); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace rp

// Access-record generation and the digit histograms of every sort pass.
//
// One work item writes a contiguous run of records: either one block's
// accesses over a range of points (same-block view, block-major order) or
// one point's accesses over a range of blocks (cross-block view,
// point-major order).  Each record is a pure function of (point, block,
// thread): the word is (a*tid + b*bid + c) mod words (Euclidean residue),
// and the executing threads are those with tid % m == r.  While writing,
// every item counts the radix digits of all sort passes in LDS and stores
// the counts to its own row of a histogram table; hist_scan_kernel sums the
// rows of a sort segment and turns them into each pass's digit offsets.
#include "common.h"
#include "launch.h"

namespace rp {

constexpr int GEN_BLOCK = 256;

template <int RB>
__device__ __forceinline__ void count_digits(uint32_t* hist, uint64_t rec, int shift,
                                             int passes, bool valid) {
  constexpr uint32_t R = 1u << RB;
  const uint64_t act = __ballot(valid);
  if (!valid) return;
  const int first = __ffsll((unsigned long long)act) - 1;
  for (int p = 0; p < passes; p++) {
    const uint32_t d = digit_at(rec, shift + p * RB, R - 1);
    const uint32_t d0 = __shfl(d, first);
    // all active lanes on one digit (the usual case for the high digits):
    // one LDS add for the wave
    const uint64_t same = __ballot(d == d0);
    if (same == act) {
      if ((int)__lane_id() == first) atomicAdd(&hist[p * R + d], (uint32_t)__popcll(act));
    } else {
      atomicAdd(&hist[p * R + d], 1u);
    }
  }
}

template <int RB>
__global__ __launch_bounds__(GEN_BLOCK) void gen_kernel(const GenItem* __restrict__ items,
                                                        const Job* __restrict__ jobs,
                                                        const SortSeg* __restrict__ segs,
                                                        uint64_t* __restrict__ recs,
                                                        uint32_t* __restrict__ item_hist,
                                                        int passes) {
  constexpr uint32_t R = 1u << RB;
  __shared__ uint32_t hist[MAX_SORT_PASSES * R];
  __shared__ uint32_t s_i;
  const GenItem it = items[blockIdx.x];
  const Job& J = jobs[it.job];
  const SortSeg sg = segs[it.seg];
  const int shift = (int)sg.shift;
  uint64_t* out = recs + sg.beg;
  for (uint32_t q = threadIdx.x; q < (uint32_t)passes * R; q += GEN_BLOCK) hist[q] = 0;
  const uint32_t ks = J.key_shift, tb = J.tbits, bb = J.bbits, pb = J.pbits, nb = J.nbits;
  const uint32_t P = J.P;
  // first point of the item: largest i with prefix[i] <= offset
  const uint64_t* pre = it.view == 0 ? J.cnt_pre : J.gcnt_pre;
  const uint64_t scale = it.view == 0 ? 1 : J.B;
  uint64_t first = it.view == 0 ? it.o0 % J.rblk : it.o0;
  if (threadIdx.x == 0) {
    uint32_t lo = 0, hi = P - 1;
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (pre[mid] * scale <= first) lo = mid; else hi = mid - 1;
    }
    s_i = lo;
  }
  __syncthreads();
  uint32_t i = s_i;
  uint64_t pos = it.o0;
  if (it.view == 0) {
    // block-major: block k, points in order, executing threads in order
    uint32_t k = (uint32_t)(it.o0 / J.rblk);
    uint64_t u0 = first - pre[i];
    while (pos < it.o1) {
      const uint64_t c = pre[i + 1] - pre[i];
      const uint64_t take = (c - u0) < (it.o1 - pos) ? (c - u0) : (it.o1 - pos);
      if (take) {
        const DPoint p = J.pts[i];
        const uint64_t arr = (uint64_t)p.array << nb;
        const uint64_t low = ((uint64_t)k << (pb + tb)) | ((uint64_t)i << tb);
        for (uint64_t q0 = 0; q0 < take; q0 += GEN_BLOCK) {
          const uint64_t q = q0 + threadIdx.x;
          const bool valid = q < take;
          uint64_t rec = 0;
          if (valid) {
            const uint32_t t = p.r + p.m * (uint32_t)(u0 + q);
            rec = ((arr | word_of(p, t, k)) << ks) | low | t;
            out[pos + q] = rec;
          }
          count_digits<RB>(hist, rec, shift, passes, valid);
        }
      }
      pos += take;
      u0 = 0;
      if (++i == P) { i = 0; k++; }
    }
  } else {
    // point-major over GLOBAL access points: point i, blocks in order,
    // executing threads in order
    uint64_t j0 = first - pre[i] * J.B;
    while (pos < it.o1) {
      const uint64_t c = pre[i + 1] - pre[i];
      const uint64_t span = c * J.B;
      const uint64_t take = (span - j0) < (it.o1 - pos) ? (span - j0) : (it.o1 - pos);
      if (take) {
        const DPoint p = J.pts[i];
        const uint32_t cnt = (uint32_t)c;
        const uint64_t arr = (uint64_t)p.array << nb;
        const uint64_t pf = (uint64_t)i << (bb + tb);
        for (uint64_t q0 = 0; q0 < take; q0 += GEN_BLOCK) {
          const uint64_t q = q0 + threadIdx.x;
          const bool valid = q < take;
          uint64_t rec = 0;
          if (valid) {
            const uint64_t j = j0 + q;
            const uint32_t kk = (uint32_t)(j / cnt);
            const uint32_t u = (uint32_t)(j - (uint64_t)kk * cnt);
            const uint32_t t = p.r + p.m * u;
            rec = ((arr | word_of(p, t, kk)) << ks) | pf | ((uint64_t)kk << tb);
            out[pos + q] = rec;
          }
          count_digits<RB>(hist, rec, shift, passes, valid);
        }
      }
      pos += take;
      j0 = 0;
      i++;
    }
  }
  __syncthreads();
  uint32_t* row = item_hist + (size_t)blockIdx.x * passes * R;
  for (uint32_t q = threadIdx.x; q < (uint32_t)passes * R; q += GEN_BLOCK) row[q] = hist[q];
}

// Block-wide exclusive scan of 64-bit values over 256 threads.
__device__ __forceinline__ uint64_t block_excl_scan256(uint64_t v, uint64_t* sm, uint64_t* total) {
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  uint64_t inc = v;
  for (int off = 1; off < 64; off <<= 1) {
    uint64_t y = __shfl_up(inc, off);
    if (lane >= off) inc += y;
  }
  if (lane == 63) sm[w] = inc;
  __syncthreads();
  uint64_t pre = 0, tot = 0;
  for (int q = 0; q < 4; q++) {
    if (q < w) pre += sm[q];
    tot += sm[q];
  }
  __syncthreads();
  *total = tot;
  return pre + inc - v;
}

// One workgroup per (segment, pass): digit totals over the segment's items,
// exclusive scan over digits, offset by the segment's first record.
template <int RB>
__global__ __launch_bounds__(256) void hist_scan_kernel(const uint32_t* __restrict__ item_hist,
                                                        const uint32_t* __restrict__ seg_item_beg,
                                                        const SortSeg* __restrict__ segs,
                                                        int passes, uint64_t* __restrict__ dbase) {
  constexpr uint32_t R = 1u << RB;
  constexpr uint32_t PER = R / 256;   // digits per thread (R >= 256)
  __shared__ uint64_t sm[4];
  const uint32_t seg = blockIdx.x / passes, p = blockIdx.x % passes;
  const uint32_t i0 = seg_item_beg[seg], i1 = seg_item_beg[seg + 1];
  uint64_t cnt[PER];
  uint64_t local = 0;
  for (uint32_t q = 0; q < PER; q++) {
    const uint32_t d = threadIdx.x * PER + q;
    uint64_t s = 0;
    for (uint32_t it = i0; it < i1; it++) s += item_hist[((size_t)it * passes + p) * R + d];
    cnt[q] = s;
    local += s;
  }
  uint64_t total;
  uint64_t run = block_excl_scan256(local, sm, &total) + segs[seg].beg;
  uint64_t* out = dbase + ((size_t)seg * passes + p) * R;
  for (uint32_t q = 0; q < PER; q++) {
    out[threadIdx.x * PER + q] = run;
    run += cnt[q];
  }
}

hipError_t launch_gen(int rb, const GenItem* items, uint32_t n_items, const Job* jobs,
                      const SortSeg* segs, uint64_t* recs, uint32_t* item_hist, int passes,
                      hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  switch (rb) {
    case 8: gen_kernel<8><<<n_items, GEN_BLOCK, 0, s>>>(items, jobs, segs, recs, item_hist, passes); break;
    case 9: gen_kernel<9><<<n_items, GEN_BLOCK, 0, s>>>(items, jobs, segs, recs, item_hist, passes); break;
    case 10: gen_kernel<10><<<n_items, GEN_BLOCK, 0, s>>>(items, jobs, segs, recs, item_hist, passes); break;
    case 11: gen_kernel<11><<<n_items, GEN_BLOCK, 0, s>>>(items, jobs, segs, recs, item_hist, passes); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_hist_scan(int rb, const uint32_t* item_hist, const uint32_t* seg_item_beg,
                            const SortSeg* segs, uint32_t nseg, int passes, uint64_t* dbase,
                            hipStream_t s) {
  if (nseg == 0 || passes == 0) return hipSuccess;
  const uint32_t g = nseg * passes;
  switch (rb) {
    case 8: hist_scan_kernel<8><<<g, 256, 0, s>>>(item_hist, seg_item_beg, segs, passes, dbase); break;
    case 9: hist_scan_kernel<9><<<g, 256, 0, s>>>(item_hist, seg_item_beg, segs, passes, dbase); break;
    case 10: hist_scan_kernel<10><<<g, 256, 0, s>>>(item_hist, seg_item_beg, segs, passes, dbase); break;
    case 11: hist_scan_kernel<11><<<g, 256, 0, s>>>(item_hist, seg_item_beg, segs, passes, dbase); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace rp

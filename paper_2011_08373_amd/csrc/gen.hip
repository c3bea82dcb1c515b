// Access-record generation.
//
// One work item writes a contiguous run of records of one log: the
// same-block log in block-major order, the cross-block log (GLOBAL arrays
// only) in point-major order; common.h describes the packing.  Each record
// is a pure function of (point, block, thread): the word is
// (a*tid + b*bid + c) mod words (Euclidean residue), and the executing
// threads are those with tid % m == r.  Items coincide with the sort's
// chunks: while writing, an item counts the radix digits of the first sort
// pass in LDS and stores them as its chunk's count row.  The item's points
// (up to 256, from its first point on) are staged in LDS first.
#include "common.h"
#include "launch.h"

namespace rp {

constexpr int GEN_BLOCK = 256;
constexpr uint32_t GEN_CACHE = 256;   // points staged in LDS per item

template <int RB>
__device__ __forceinline__ void count_digits(uint32_t* hist, uint64_t rec, int shift, bool valid) {
  constexpr uint32_t R = 1u << RB;
  // the valid lanes of a call are a prefix of the wave: lane 0 is the first
  const uint64_t act = __ballot(valid);
  if (!act) return;
  const uint32_t d = digit_at(rec, shift, R - 1);
  const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
  if (!valid) return;
  const int first = 0;
  // all active lanes on one digit (the usual case for the high digits):
  // one LDS add for the wave
  const uint64_t same = __ballot(d == d0);
  if (same == act) {
    if ((int)__lane_id() == first) atomicAdd(&hist[d], (uint32_t)__popcll(act));
  } else {
    atomicAdd(&hist[d], 1u);
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
  __shared__ uint32_t hist[R];
  __shared__ DPoint s_pts[GEN_CACHE];        // points i0, i0+1, ... (mod P) of the item
  __shared__ uint64_t s_cnt[GEN_CACHE];      // their records (per block in the same-block log)
  __shared__ uint32_t s_i;
  const GenItem it = items[blockIdx.x];
  const Job& J = jobs[it.job];
  const SortSeg sg = segs[it.seg];
  const int shift = (int)sg.shift;
  const int count = passes > 0;
  uint64_t* out = recs + sg.beg;
  for (uint32_t q = threadIdx.x; q < R; q += GEN_BLOCK) hist[q] = 0;
  const uint32_t ks = J.key_shift, tb = J.tbits, bb = J.bbits, pb = J.pbits, nb = J.nbits;
  const uint32_t P = J.P;
  // first point of the item: largest i with prefix[i] <= offset
  const uint64_t* pre = it.view == 0 ? J.cnt_pre : J.gcnt_pre;
  const uint64_t first = it.view == 0 ? it.o0 % J.rblk : it.o0;
  if (threadIdx.x == 0) {
    uint32_t lo = 0, hi = P - 1;
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (pre[mid] <= first) lo = mid; else hi = mid - 1;
    }
    s_i = lo;
  }
  __syncthreads();
  const uint32_t i0 = s_i;
  const uint32_t nc = P < GEN_CACHE ? P : GEN_CACHE;
  for (uint32_t d = threadIdx.x; d < nc; d += GEN_BLOCK) {
    uint32_t i = i0 + d;
    if (i >= P) i -= P;
    s_pts[d] = J.pts[i];
    s_cnt[d] = pre[i + 1] - pre[i];
  }
  __syncthreads();
  uint32_t i = i0;
  uint32_t d = 0;            // cache slot of point i (i0 + d mod P)
  uint64_t pos = it.o0;
  if (it.view == 0) {
    // block-major: block k, points in order, executing threads in order
    uint32_t k = (uint32_t)(it.o0 / J.rblk);
    uint64_t u0 = first - pre[i];
    while (pos < it.o1) {
      const bool cached = d < nc;
      const uint64_t c = cached ? s_cnt[d] : pre[i + 1] - pre[i];
      const uint64_t take = (c - u0) < (it.o1 - pos) ? (c - u0) : (it.o1 - pos);
      if (take) {
        const DPoint p = cached ? s_pts[d] : J.pts[i];
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
          if (count) count_digits<RB>(hist, rec, shift, valid);
        }
      }
      pos += take;
      u0 = 0;
      d++;
      if (++i == P) { i = 0; k++; }
    }
  } else {
    // point-major over GLOBAL access points: point i, blocks in order,
    // executing threads in order (one thread when the word does not depend
    // on it; blocks 0 and 1 only when it does not depend on the block)
    uint64_t j0 = first - pre[i];
    while (pos < it.o1) {
      const bool cached = d < nc;
      const uint64_t span = cached ? s_cnt[d] : pre[i + 1] - pre[i];
      const uint64_t take = (span - j0) < (it.o1 - pos) ? (span - j0) : (it.o1 - pos);
      if (take) {
        const DPoint p = cached ? s_pts[d] : J.pts[i];
        const uint32_t cnt = (p.flags & PF_TCONST) ? 1u : p.cnt;
        const uint64_t arr = (uint64_t)p.array << nb;
        const uint64_t pf = (uint64_t)i << (bb + tb);
        for (uint64_t q0 = 0; q0 < take; q0 += GEN_BLOCK) {
          const uint64_t q = q0 + threadIdx.x;
          const bool valid = q < take;
          uint64_t rec = 0;
          if (valid) {
            const uint64_t j = j0 + q;
            uint32_t kk, u;
            if (span < (1ull << 32)) {
              kk = (uint32_t)j / cnt;
              u = (uint32_t)j - kk * cnt;
            } else {
              kk = (uint32_t)(j / cnt);
              u = (uint32_t)(j - (uint64_t)kk * cnt);
            }
            const uint32_t t = p.r + p.m * u;
            rec = ((arr | word_of(p, t, kk)) << ks) | pf | ((uint64_t)kk << tb);
            out[pos + q] = rec;
          }
          if (count) count_digits<RB>(hist, rec, shift, valid);
        }
      }
      pos += take;
      j0 = 0;
      d++;
      i++;
    }
  }
  if (!count) return;
  __syncthreads();
  uint32_t* row = item_hist + (size_t)blockIdx.x * R;
  for (uint32_t q = threadIdx.x; q < R; q += GEN_BLOCK) row[q] = hist[q];
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

}  // namespace rp

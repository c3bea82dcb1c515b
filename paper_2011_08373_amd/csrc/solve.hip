// Solve of Alg. 1: the minimum-weight barrier assignment satisfying phi
// (weighted partial MaxSAT with phi hard and {not b_s} soft, Sections 2.3-2.4),
// ties broken by (number of enabled barriers, mask as an unsigned integer).
// As one integer the key is the sum over enabled slots of
// w_s*2^71 + 2^64 + 2^s, so it is additive over slots and the optimum is
// unique.  It is carried as (hi, lo) = (sum of w_s*128+1, mask).
//
// Under the mhs strategy the rounds before the first SAFE take the greedy
// hitting set of greedy_solve instead, and the round after it the exact
// query (phase PH_FINAL) that confirms or replaces the greedy answer.
//
// One workgroup per job:
//   1. unit propagation: positive units force a slot on, negative units
//      force it off, a clause with no literal left proves UNSAT; a slot that
//      is in no positive literal of an open clause is set off (it can only
//      add weight);
//   2. the open clauses split into components over the free slots (the key
//      is additive, so components are solved independently);
//   3. a component of k <= 20 slots is enumerated bit-sliced: a 64-bit word
//      holds the six lowest slots' 64 assignments, every clause is evaluated
//      on whole words with AND/OR, and each word's cheapest feasible pattern
//      is found through the patterns pre-sorted by key;
//   4. a wider component is searched depth-first by all waves of the
//      workgroup: branch on the free positive literals of the open clause
//      with the fewest of them, prune on key and on a per-clause lower bound;
//      clause tests are spread over the 64 lanes and combined with
//      cross-lane reductions.  The tree's nodes at depth SPLIT_DEPTH are
//      dealt out to the waves in the order of the search (every wave walks
//      the levels above it alike, pruning there only dead nodes, so they all
//      number those nodes the same way); below it each wave searches its own
//      subtrees, pruning against the smallest weight any wave has found so
//      far (a shared word) as well as its own best key.  The optimum is
//      unique, so the smallest of the waves' best keys is the answer whatever
//      order the waves run in.
#include "common.h"
#include "launch.h"

namespace rp {

constexpr int SV_BLOCK = 256;
constexpr int SV_WAVES = SV_BLOCK / 64;
constexpr uint32_t SV_LDS_CLAUSES = 3072;
constexpr int ENUM_MAX = 20;

struct Key { uint64_t hi, lo; };
__device__ __forceinline__ bool key_lt(Key a, Key b) { return a.hi != b.hi ? a.hi < b.hi : a.lo < b.lo; }

template <typename T>
__device__ __forceinline__ T wave_or(T v) {
  for (int off = 32; off > 0; off >>= 1) v |= __shfl_xor(v, off);
  return v;
}
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
  for (int off = 32; off > 0; off >>= 1) {
    uint64_t o = __shfl_xor(v, off);
    v = o < v ? o : v;
  }
  return v;
}
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
  for (int off = 32; off > 0; off >>= 1) {
    uint64_t o = __shfl_xor(v, off);
    v = o > v ? o : v;
  }
  return v;
}

__device__ __forceinline__ uint64_t block_or(uint64_t v, uint64_t* sm) {
  v = wave_or(v);
  const int w = threadIdx.x >> 6;
  if (__lane_id() == 0) sm[w] = v;
  __syncthreads();
  uint64_t r = 0;
  for (int q = 0; q < SV_WAVES; q++) r |= sm[q];
  __syncthreads();
  return r;
}

__device__ __forceinline__ Key block_min_key(Key k, uint64_t* smh, uint64_t* sml) {
  for (int off = 32; off > 0; off >>= 1) {
    Key o;
    o.hi = __shfl_xor(k.hi, off);
    o.lo = __shfl_xor(k.lo, off);
    if (key_lt(o, k)) k = o;
  }
  const int w = threadIdx.x >> 6;
  if (__lane_id() == 0) { smh[w] = k.hi; sml[w] = k.lo; }
  __syncthreads();
  Key r = {smh[0], sml[0]};
  for (int q = 1; q < SV_WAVES; q++) {
    Key o = {smh[q], sml[q]};
    if (key_lt(o, r)) r = o;
  }
  __syncthreads();
  return r;
}

// pattern of local slot b (< 6) over the 64 assignments of a word
__device__ __forceinline__ uint64_t pat(int b) {
  const uint64_t P6[6] = {0xAAAAAAAAAAAAAAAAull, 0xCCCCCCCCCCCCCCCCull, 0xF0F0F0F0F0F0F0F0ull,
                          0xFF00FF00FF00FF00ull, 0xFFFF0000FFFF0000ull, 0xFFFFFFFF00000000ull};
  return P6[b];
}

struct DfsFrame { uint64_t ones, zeros, khi, klo, todo, tried; };
constexpr int SPLIT_DEPTH = 3;           // depth whose nodes are dealt out to the waves

constexpr uint32_t GREEDY_MAX = 16384;   // clauses the greedy step handles (bitset in LDS)

// The mhs strategy's Solve (Section 2.4): the greedy minimal hitting set of
// the positive clauses of phi -- repeatedly the slot hitting the most clauses
// not yet hit per unit of weight (exact integer comparison, ties to the lower
// slot), then every pick whose removal leaves all positive clauses hit is
// dropped, last pick first.  Returns false (the caller solves exactly) when
// phi has an empty clause, is too long, or the set breaks a clause of phi.
__device__ bool greedy_solve(const Job& J, JobState* st, uint32_t n, const rp_clause* C,
                             uint32_t* s_hit, uint32_t* s_c64, uint32_t* s_pick,
                             uint32_t* s_best, uint64_t* sm) {
  const int tid = threadIdx.x;
  const uint32_t S = J.S;
  if (n > GREEDY_MAX) return false;
  const uint32_t nw = (n + 31) / 32;
  for (uint32_t q = tid; q < nw; q += SV_BLOCK) s_hit[q] = 0;
  __syncthreads();
  uint64_t bad = 0;
  for (uint32_t q = tid; q < n; q += SV_BLOCK) {
    const rp_clause c = C[q];
    if (c.pos == 0 && c.neg == 0) bad = 1;
    if (!(c.pos && !c.neg)) atomicOr(&s_hit[q >> 5], 1u << (q & 31));   // not positive: ignored
  }
  if (block_or(bad, sm)) return false;
  uint64_t x = 0;
  uint32_t np = 0;
  for (uint32_t it = 0; it < 64; it++) {
    if (tid < 64) s_c64[tid] = 0;
    __syncthreads();
    for (uint32_t q = tid; q < n; q += SV_BLOCK) {
      if ((s_hit[q >> 5] >> (q & 31)) & 1) continue;
      uint64_t p = C[q].pos;
      while (p) {
        const uint32_t b = __ffsll((unsigned long long)p) - 1;
        p &= p - 1;
        atomicAdd(&s_c64[b], 1u);
      }
    }
    __syncthreads();
    if (tid == 0) {
      int best = -1;
      for (uint32_t b = 0; b < S; b++) {
        if (!s_c64[b]) continue;
        if (best < 0 || (uint64_t)s_c64[b] * J.weights[best] > (uint64_t)s_c64[best] * J.weights[b])
          best = (int)b;
      }
      *s_best = best < 0 ? NONE32 : (uint32_t)best;
      if (best >= 0) s_pick[np] = (uint32_t)best;
    }
    __syncthreads();
    const uint32_t b = *s_best;
    if (b == NONE32) break;
    x |= 1ull << b;
    np++;
    for (uint32_t q = tid; q < n; q += SV_BLOCK)
      if (!((s_hit[q >> 5] >> (q & 31)) & 1) && ((C[q].pos >> b) & 1))
        atomicOr(&s_hit[q >> 5], 1u << (q & 31));
    __syncthreads();
  }
  for (int k = (int)np - 1; k >= 0; k--) {
    const uint64_t y = x & ~(1ull << s_pick[k]);
    uint64_t miss = 0;
    for (uint32_t q = tid; q < n; q += SV_BLOCK) {
      const rp_clause c = C[q];
      if (c.pos && !c.neg && !(c.pos & y)) miss = 1;
    }
    if (!block_or(miss, sm)) x = y;
  }
  uint64_t viol = 0;
  for (uint32_t q = tid; q < n; q += SV_BLOCK) {
    const rp_clause c = C[q];
    if (!((c.pos & x) || (c.neg & ~x))) viol = 1;
  }
  if (block_or(viol, sm)) return false;
  if (tid == 0) {
    uint64_t W = 0;
    for (uint32_t b = 0; b < S; b++)
      if ((x >> b) & 1) W += J.weights[b];
    st->x = x;
    st->weight = W;
    if (st->max_rounds && st->rounds >= st->max_rounds) st->state = ST_ROUNDS;
  }
  return true;
}

__global__ __launch_bounds__(SV_BLOCK) void solve_kernel(const Job* __restrict__ jobs) {
  __shared__ rp_clause s_cl[SV_LDS_CLAUSES];    // open clauses (restricted), 48 KiB
  __shared__ uint64_t s_lp[SV_LDS_CLAUSES / 2];  // per component: local pos / neg / aux
  __shared__ uint64_t s_ln[SV_LDS_CLAUSES / 2];
  __shared__ uint64_t s_la[SV_LDS_CLAUSES / 2];
  __shared__ uint64_t s_kh[64], s_kl[64];        // local slot key parts
  __shared__ uint64_t s_lowh[64], s_lowl[64];    // key of each low pattern
  __shared__ uint32_t s_order[64];
  __shared__ uint32_t s_gslot[64];
  __shared__ uint64_t smA[SV_WAVES], smB[SV_WAVES];
  __shared__ uint32_t s_cnt;
  __shared__ DfsFrame s_stack[SV_WAVES][65];
  __shared__ unsigned long long s_bound;         // smallest weight part found by any wave
  __shared__ uint32_t s_overflow;
  __shared__ uint64_t s_inch[SV_WAVES], s_incl[SV_WAVES];
  __shared__ uint32_t s_hit[GREEDY_MAX / 32];
  __shared__ uint32_t s_c64[64], s_pick[64], s_best;

  const Job& J = jobs[blockIdx.x];
  JobState* st = J.st;
  if (st->state != ST_RUN) return;
  const int tid = threadIdx.x, lane = __lane_id(), wv = tid >> 6;
  const uint32_t S = J.S;
  const uint64_t all = S >= 64 ? ~0ull : ((1ull << S) - 1);
  const uint32_t n = st->n_phi;
  const rp_clause* C = J.phi;
  const uint32_t phase = st->phase;
  if (phase == PH_GREEDY && greedy_solve(J, st, n, C, s_hit, s_c64, s_pick, &s_best, smA)) return;

  // ---- 1. propagation
  uint64_t on = 0, off = 0;
  bool unsat = false;
  for (int iter = 0; iter < 200; iter++) {
    uint64_t non = 0, noff = 0, core = 0, bad = 0;
    for (uint32_t q = tid; q < n; q += SV_BLOCK) {
      const rp_clause c = C[q];
      if ((c.pos & on) || (c.neg & off)) continue;
      const uint64_t p = c.pos & ~off, m = c.neg & ~on;
      if (p == 0 && m == 0) bad = 1;
      else if (p == 0 && __popcll(m) == 1) noff |= m;
      else if (m == 0 && __popcll(p) == 1) non |= p;
      core |= p;
    }
    non = block_or(non, smA);
    noff = block_or(noff, smA);
    core = block_or(core, smA);
    bad = block_or(bad, smA);
    if (bad || (non & (off | noff)) || (noff & (on | non))) { unsat = true; break; }
    const uint64_t nz = all & ~on & ~off & ~non & ~noff & ~core;
    if ((non | noff | nz) == 0) break;
    on |= non;
    off |= noff | nz;
  }
  if (unsat) {
    if (tid == 0) st->state = ST_UNSAT;
    return;
  }
  const uint64_t freeS = all & ~on & ~off;

  // ---- open clauses restricted to the free slots
  if (tid == 0) s_cnt = 0;
  __syncthreads();
  rp_clause* U = s_cl;
  const bool lds = n <= SV_LDS_CLAUSES;
  if (!lds) U = J.scratch;   // scratch holds >= n clauses
  for (uint32_t q = tid; q < n; q += SV_BLOCK) {
    const rp_clause c = C[q];
    if ((c.pos & on) || (c.neg & off)) continue;
    rp_clause r;
    r.pos = c.pos & freeS;
    r.neg = c.neg & freeS;
    U[atomicAdd(&s_cnt, 1u)] = r;
  }
  __syncthreads();
  const uint32_t nu = s_cnt;

  uint64_t result = on;
  uint64_t left = freeS;
  while (left) {
    // ---- 2. component of the lowest free slot
    uint64_t comp = left & (~left + 1);
    for (;;) {
      uint64_t add = 0;
      for (uint32_t q = tid; q < nu; q += SV_BLOCK) {
        const uint64_t l = U[q].pos | U[q].neg;
        if ((l & comp) && (l & ~comp)) add |= l;
      }
      add = block_or(add, smA);
      if (add == 0 || (add & ~comp) == 0) break;
      comp |= add;
    }
    left &= ~comp;
    const int k = __popcll(comp);
    // local slot numbering
    if (tid == 0) {
      uint64_t m = comp;
      int b = 0;
      while (m) {
        const uint32_t s = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        s_gslot[b] = s;
        s_kh[b] = (uint64_t)J.weights[s] * 128u + 1u;
        s_kl[b] = 1ull << s;
        b++;
      }
      s_cnt = 0;
    }
    __syncthreads();
    // component clauses in local numbering (s_lp/s_ln), aux = lower bound
    const uint32_t cap_local = SV_LDS_CLAUSES / 2;
    for (uint32_t q = tid; q < nu; q += SV_BLOCK) {
      const rp_clause c = U[q];
      if (!((c.pos | c.neg) & comp)) continue;
      uint64_t lp = 0, ln = 0, lb = ~0ull;
      for (int b = 0; b < k; b++) {
        const uint64_t g = 1ull << s_gslot[b];
        if (c.pos & g) { lp |= 1ull << b; lb = s_kh[b] < lb ? s_kh[b] : lb; }
        if (c.neg & g) ln |= 1ull << b;
      }
      const uint32_t slot = atomicAdd(&s_cnt, 1u);
      if (slot < cap_local) { s_lp[slot] = lp; s_ln[slot] = ln; s_la[slot] = lp ? lb : 0; }
    }
    __syncthreads();
    const uint32_t nc = s_cnt;
    if (nc > cap_local) {
      if (tid == 0) { st->err = ERR_SCRATCH; st->state = ST_ERROR; }
      return;
    }
    Key best = {~0ull, ~0ull};
    if (k <= ENUM_MAX) {
      // ---- 3. bit-sliced enumeration
      const int low = k < 6 ? k : 6;
      if (tid < 64) {
        uint64_t h = 0, l = 0;
        for (int b = 0; b < low; b++)
          if ((tid >> b) & 1) { h += s_kh[b]; l |= s_kl[b]; }
        s_lowh[tid] = h;
        s_lowl[tid] = l;
      }
      __syncthreads();
      if (tid < 64) {   // rank of pattern tid by key
        uint32_t rk = 0;
        const Key me = {s_lowh[tid], s_lowl[tid]};
        for (int o = 0; o < 64; o++) {
          const Key ot = {s_lowh[o], s_lowl[o]};
          if (key_lt(ot, me) || (ot.hi == me.hi && ot.lo == me.lo && o < tid)) rk++;
        }
        s_order[rk] = tid;
      }
      __syncthreads();
      const uint64_t valid = low == 6 ? ~0ull : ((1ull << (1u << low)) - 1);
      const uint32_t nwords = 1u << (k - low);
      const uint64_t lowmask = (1ull << low) - 1;
      for (uint32_t H = tid; H < nwords; H += SV_BLOCK) {
        uint64_t feas = valid;
        const uint64_t hbits = (uint64_t)H << low;
        for (uint32_t q = 0; q < nc && feas; q++) {
          const uint64_t lp = s_lp[q], ln = s_ln[q];
          uint64_t sp, sn;
          if (lp & hbits) sp = ~0ull;
          else {
            sp = 0;
            uint64_t m = lp & lowmask;
            while (m) { const int b = __ffsll((unsigned long long)m) - 1; m &= m - 1; sp |= pat(b); }
          }
          if (ln & ~hbits & ~lowmask) sn = ~0ull;
          else {
            sn = 0;
            uint64_t m = ln & lowmask;
            while (m) { const int b = __ffsll((unsigned long long)m) - 1; m &= m - 1; sn |= ~pat(b); }
          }
          feas &= sp | sn;
        }
        if (!feas) continue;
        Key kh = {0, 0};
        uint64_t m = hbits;
        while (m) {
          const int b = __ffsll((unsigned long long)m) - 1;
          m &= m - 1;
          kh.hi += s_kh[b];
          kh.lo |= s_kl[b];
        }
        for (int o = 0; o < 64; o++) {
          const uint32_t pt = s_order[o];
          if ((feas >> pt) & 1) {
            const Key cand = {kh.hi + s_lowh[pt], kh.lo | s_lowl[pt]};
            if (key_lt(cand, best)) best = cand;
            break;
          }
        }
      }
      best = block_min_key(best, smA, smB);
    } else {
      // ---- 4. depth-first branch and bound by every wave
      if (tid == 0) {
        s_bound = ~0ull;
        s_overflow = 0;
      }
      __syncthreads();
      {
        DfsFrame* stk = s_stack[wv];
        Key inc = {~0ull, ~0ull};
        bool found = false;
        uint64_t nodes = 0;
        uint32_t split_idx = 0;      // nodes met at SPLIT_DEPTH so far
        int depth = 0;
        // a frame is pushed only after its node was evaluated: todo holds
        // the free literals of the chosen open clause
        uint64_t ones = 0, zeros = 0;
        Key key = {0, 0};
        bool eval_pending = true;
        bool overflow = false;
        while (true) {
          if (eval_pending) {
            eval_pending = false;
            bool mine = true;
            if (depth == SPLIT_DEPTH) mine = (split_idx++ % SV_WAVES) == (uint32_t)wv;
            // above the split every wave evaluates every node alike (no
            // bound pruning there, so the numbering agrees); below it a node
            // no better than a known weight is skipped
            const uint64_t bound = depth >= SPLIT_DEPTH
                                       ? (uint64_t)__hip_atomic_load(&s_bound, __ATOMIC_RELAXED,
                                                                     __HIP_MEMORY_SCOPE_WORKGROUP)
                                       : ~0ull;
            if (mine) nodes++;
            if (nodes > J.node_limit) { overflow = true; break; }
            const bool skip = !mine || (depth >= SPLIT_DEPTH &&
                                        ((found && !key_lt(key, inc)) || key.hi > bound));
            if (!skip) {
              uint64_t dead = 0, pick = ~0ull, lbmax = 0;
              for (uint32_t q = lane; q < nc; q += 64) {
                const uint64_t lp = s_lp[q], ln = s_ln[q];
                if ((lp & ones) || (ln & ~ones)) continue;   // satisfied with undecided = 0
                const uint64_t fr = lp & ~zeros;
                if (fr == 0) { dead = 1; continue; }
                const uint64_t cand = ((uint64_t)__popcll(fr) << 32) | q;
                pick = cand < pick ? cand : pick;
                lbmax = s_la[q] > lbmax ? s_la[q] : lbmax;
              }
              dead = wave_or(dead);
              pick = wave_min_u64(pick);
              lbmax = wave_max_u64(lbmax);
              if (!dead) {
                if (pick == ~0ull) {
                  // every clause holds: a solution
                  if (!found || key_lt(key, inc)) {
                    inc = key;
                    found = true;
                    if (lane == 0)
                      __hip_atomic_fetch_min(&s_bound, (unsigned long long)key.hi,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                  }
                } else if (depth < SPLIT_DEPTH ||
                           !((found && key.hi + lbmax > inc.hi) || key.hi + lbmax > bound)) {
                  const uint32_t q = (uint32_t)(pick & 0xFFFFFFFFu);
                  // every lane writes the same frame, so each lane's later
                  // read follows its own write
                  DfsFrame f;
                  f.ones = ones; f.zeros = zeros; f.khi = key.hi; f.klo = key.lo;
                  f.todo = s_lp[q] & ~zeros; f.tried = 0;
                  stk[depth] = f;
                  __builtin_amdgcn_wave_barrier();
                  depth++;
                }
              }
            }
          }
          // next branch of the deepest frame with literals left
          if (depth == 0) break;
          __builtin_amdgcn_wave_barrier();
          DfsFrame f = stk[depth - 1];
          if (f.todo == 0) { depth--; continue; }
          const uint64_t sbit = f.todo & (~f.todo + 1);
          const int b = __ffsll((unsigned long long)sbit) - 1;
          __builtin_amdgcn_wave_barrier();
          stk[depth - 1].todo = f.todo & ~sbit;
          stk[depth - 1].tried = f.tried | sbit;
          __builtin_amdgcn_wave_barrier();
          ones = f.ones | sbit;
          zeros = f.zeros | f.tried;
          key.hi = f.khi + s_kh[b];
          key.lo = f.klo | s_kl[b];
          eval_pending = true;
        }
        if (lane == 0) {
          if (overflow) atomicOr(&s_overflow, 1u);
          s_inch[wv] = found ? inc.hi : ~0ull;
          s_incl[wv] = found ? inc.lo : ~0ull;
        }
      }
      __syncthreads();
      if (s_overflow) {
        if (tid == 0) { st->err = ERR_NODES; st->state = ST_ERROR; }
        return;
      }
      best.hi = s_inch[0];
      best.lo = s_incl[0];
      for (int q = 1; q < SV_WAVES; q++) {
        const Key o = {s_inch[q], s_incl[q]};
        if (key_lt(o, best)) best = o;
      }
      __syncthreads();
    }
    if (best.hi == ~0ull && best.lo == ~0ull) {
      if (tid == 0) st->state = ST_UNSAT;
      return;
    }
    result |= best.lo;   // lo is the global mask of the component's optimum
    __syncthreads();
  }
  if (tid == 0) {
    uint64_t W = 0;
    for (uint32_t s = 0; s < S; s++)
      if ((result >> s) & 1) W += J.weights[s];
    if (phase == PH_FINAL) {
      // the exact query after the greedy answer was verified SAFE
      st->phase = PH_EXACT;
      if (result == st->x) {
        st->weight = W;
        st->state = ST_SAFE;
        return;
      }
    }
    st->x = result;
    st->weight = W;
    if (st->max_rounds && st->rounds >= st->max_rounds) st->state = ST_ROUNDS;
  }
}

hipError_t launch_solve(const Job* jobs, uint32_t njobs, hipStream_t s) {
  if (njobs == 0) return hipSuccess;
  solve_kernel<<<njobs, SV_BLOCK, 0, s>>>(jobs);
  return hipGetLastError();
}

}  // namespace rp

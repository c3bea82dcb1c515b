// GenerateClause of Alg. 1 and the maintenance of the constraint set phi.
//
// One workgroup per job, after a Verify scan:
//   - counts the Verify call (and records the verified assignment);
//   - SAFE when no point has a racing partner and no enabled slot diverges;
//   - otherwise learns clauses: a race between points i < j gives the
//     positive clause of the barrier slots with an occurrence strictly
//     between i and j (grid-level slots only for a cross-block race); a
//     divergent slot s gives the negative unit {not b_s} (Section 2.4).
//     Only the first racing partner j of each point is needed: every later
//     partner's clause is a superset, hence subsumed;
//   - phi := reduce(phi + learned): sorted by (pos, neg), duplicates and
//     subsumed clauses dropped (a learned empty clause, two racing points
//     with no barrier slot between them, leaves phi = {empty} at once).  A subset precedes its supersets in that
//     order, so each clause is tested against earlier ones only.  Up to 2048
//     clauses are merged in LDS, more in the job's scratch.
#include "common.h"
#include "launch.h"

namespace rp {

constexpr int CL_BLOCK = 1024;

__device__ __forceinline__ bool cl_less(const rp_clause& a, const rp_clause& b) {
  return a.pos != b.pos ? a.pos < b.pos : a.neg < b.neg;
}

// Bitonic sort of c[0..n2) (n2 a power of two) by one workgroup.  Element i
// sits in lane i % 64 of wave (i % CL_BLOCK) / 64, so a step that pairs
// elements less than 64 apart pairs lanes of one wave.  Each merge level k
// runs its steps with a stride of 64 or more through memory (a workgroup
// barrier after each), then loads every element once and runs the steps
// with smaller strides in registers, exchanging partners by lane shuffles,
// and stores it back: the array crosses LDS once per level for those steps
// instead of once per step.
__device__ void block_bitonic(rp_clause* c, uint32_t n2) {
  const uint32_t lane = __lane_id();
  const uint32_t wbase = (threadIdx.x >> 6) * 64;
  for (uint32_t k = 2; k <= n2; k <<= 1) {
    uint32_t j = k >> 1;
    for (; j >= 64; j >>= 1) {
      for (uint32_t i = threadIdx.x; i < n2; i += CL_BLOCK) {
        const uint32_t l = i ^ j;
        if (l > i) {
          const rp_clause a = c[i], b = c[l];
          const bool up = (i & k) == 0;
          if (up ? cl_less(b, a) : cl_less(a, b)) { c[i] = b; c[l] = a; }
        }
      }
      __syncthreads();
    }
    // strides j .. 1 (j < 64) inside each wave; lanes past n2 (n2 < 64) take
    // part in the shuffles with pad values and pair only among themselves
    for (uint32_t b0 = wbase; b0 < n2; b0 += CL_BLOCK) {
      const uint32_t i = b0 + lane;
      rp_clause e;
      if (i < n2) {
        e = c[i];
      } else {
        e.pos = ~0ull;
        e.neg = ~0ull;
      }
      const bool up = (i & k) == 0;
      for (uint32_t jj = j; jj > 0; jj >>= 1) {
        rp_clause p;
        p.pos = __shfl_xor(e.pos, (int)jj);
        p.neg = __shfl_xor(e.neg, (int)jj);
        const bool lower = (i & jj) == 0;
        // the lower element of a pair keeps the smaller one on an ascending
        // run, the larger one on a descending run
        const bool take = (up == lower) ? cl_less(p, e) : cl_less(e, p);
        if (take) e = p;
      }
      if (i < n2) c[i] = e;
    }
    __syncthreads();
  }
}

__device__ __forceinline__ uint32_t block_excl_scan1024(uint32_t v, uint32_t* sm, uint32_t* total) {
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  uint32_t inc = v;
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t y = __shfl_up(inc, off);
    if (lane >= off) inc += y;
  }
  if (lane == 63) sm[w] = inc;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
  for (int q = 0; q < CL_BLOCK / 64; q++) {
    if (q < w) pre += sm[q];
    tot += sm[q];
  }
  __syncthreads();
  *total = tot;
  return pre + inc - v;
}

constexpr uint32_t CL_LDS = 2048;   // clauses merged in LDS; more go through the job's scratch
constexpr uint32_t CL_BITS = 1024;  // points whose slot bits are staged in LDS

// learn: 0 = only decide SAFE (the check call), 1 = learn and reduce.
__global__ __launch_bounds__(CL_BLOCK) void clause_kernel(const Job* __restrict__ jobs, int learn) {
  __shared__ uint32_t s_n, s_races, s_first, s_nbar, s_empty;
  __shared__ uint32_t sm[CL_BLOCK / 64];
  __shared__ uint32_t keep[4096];   // bitset over up to 131072 clauses
  __shared__ rp_clause s_cl[CL_LDS];
  // the barrier occurrences in program order (P <= CL_BITS): position,
  // slot bit (any level, grid level), and for each point the index of the
  // first occurrence at or after it
  __shared__ uint16_t s_bpos[CL_BITS];
  __shared__ uint64_t s_bbit[2][CL_BITS];
  __shared__ uint16_t s_bnext[CL_BITS + 1];
  const Job& J = jobs[blockIdx.x];
  JobState* st = J.st;
  if (st->state != ST_RUN) return;
  const int tid = threadIdx.x;
  const uint32_t P = J.P;
  const uint64_t x = st->x;
  const uint64_t div = st->divergent;
  if (tid == 0) { s_n = 0; s_races = 0; s_first = NONE32; s_empty = 0; }
  __syncthreads();
  for (uint32_t row = tid; row < 2 * P; row += CL_BLOCK) {
    if (J.minj[row] != NONE32) {
      atomicAdd(&s_races, 1u);
      atomicMin(&s_first, row);
    }
  }
  __syncthreads();
  const uint32_t races = s_races;
  if (tid == 0) {
    if (J.traj && st->rounds < J.traj_cap) J.traj[st->rounds] = x;
    st->rounds += 1;
    st->races = races;
  }
  if (races == 0 && div == 0) {
    // SAFE; under the mhs strategy the exact query still decides
    if (tid == 0) {
      if (st->phase == PH_GREEDY) st->phase = PH_FINAL;
      else st->state = ST_SAFE;
    }
    return;
  }
  if (!learn) return;
  // the slot bits between i and its partner are ORed over the barrier
  // occurrences between them (listed in LDS when the tables fit), else point
  // by point
  const bool lds_bits = P <= CL_BITS;
  if (lds_bits) {
    const uint32_t u = tid;                         // P <= CL_BITS == CL_BLOCK
    const uint64_t ba = u < P ? J.bits_any[u] : 0, bg = u < P ? J.bits_grid[u] : 0;
    uint32_t nbar;
    const uint32_t t = block_excl_scan1024(ba != 0, sm, &nbar);
    if (u < P && ba) {
      s_bpos[t] = (uint16_t)u;
      s_bbit[0][t] = ba;
      s_bbit[1][t] = bg;
    }
    if (u < P) s_bnext[u] = (uint16_t)t;
    if (tid == 0) {
      s_bnext[P] = (uint16_t)nbar;
      s_nbar = nbar;
    }
    __syncthreads();
  }
  const uint32_t nbar = lds_bits ? s_nbar : 0;
  // slot bits of the barrier occurrences strictly between points i and j
  auto between = [&](uint32_t lv, uint32_t i, uint32_t j) -> uint64_t {
    uint64_t pos = 0;
    if (lds_bits) {
      for (uint32_t t = s_bnext[i + 1]; t < nbar && s_bpos[t] < j; t++) pos |= s_bbit[lv][t];
    } else {
      const uint64_t* bits = lv ? J.bits_grid : J.bits_any;
      for (uint32_t u = i + 1; u < j; u++) pos |= bits[u];
    }
    return pos;
  };
  // phi first, then the learned clauses: in LDS when they surely fit, else
  // in the job's scratch
  const uint32_t n_phi = st->n_phi;
  const bool one = J.policy == 1;
  const uint64_t most = (uint64_t)n_phi + (one ? 1u : 2u * P + 64u);
  rp_clause* sc = most <= CL_LDS ? s_cl : J.scratch;
  for (uint32_t q = tid; q < n_phi; q += CL_BLOCK) sc[q] = J.phi[q];
  if (one) {
    if (tid == 0) {
      rp_clause c;
      if (div) {
        c.pos = 0;
        c.neg = div & (~div + 1);       // smallest divergent slot
      } else {
        const uint32_t row = s_first;   // smallest (level, i)
        const uint32_t lv = row / P, i = row % P, j = J.minj[row];
        c.pos = between(lv, i, j);
        c.neg = 0;
      }
      sc[n_phi] = c;
      s_n = 1;
    }
  } else {
    for (uint32_t row = tid; row < 2 * P; row += CL_BLOCK) {
      const uint32_t j = J.minj[row];
      if (j == NONE32) continue;
      const uint32_t lv = row / P, i = row % P;
      const uint64_t pos = between(lv, i, j);
      if (pos == 0) s_empty = 1;      // no slot between them: the empty clause
      const uint32_t slot = atomicAdd(&s_n, 1u);
      rp_clause c;
      c.pos = pos;
      c.neg = 0;
      sc[n_phi + slot] = c;
    }
    if (tid < 64 && ((div >> tid) & 1)) {
      const uint32_t slot = atomicAdd(&s_n, 1u);
      rp_clause c;
      c.pos = 0;
      c.neg = 1ull << tid;
      sc[n_phi + slot] = c;
    }
  }
  __syncthreads();
  if (s_empty) {
    // the empty clause subsumes every other: phi reduces to it alone (and
    // the next Solve proves UNSAT)
    if (tid == 0) {
      rp_clause e;
      e.pos = 0;
      e.neg = 0;
      J.phi[0] = e;
      st->n_phi = 1;
    }
    return;
  }
  const uint32_t n = n_phi + s_n;
  uint32_t n2 = 1;
  while (n2 < n) n2 <<= 1;
  if (n2 > (sc == s_cl ? CL_LDS : J.scratch_cap) || n > 4096u * 32u) {
    if (tid == 0) { st->err = ERR_SCRATCH; st->state = ST_ERROR; }
    return;
  }
  for (uint32_t q = n + tid; q < n2; q += CL_BLOCK) {
    rp_clause pad;
    pad.pos = ~0ull;
    pad.neg = ~0ull;
    sc[q] = pad;
  }
  __syncthreads();
  block_bitonic(sc, n2);
  // keep = first of its duplicates and not a strict superset of an earlier clause
  for (uint32_t q = tid; q < (n + 31) / 32; q += CL_BLOCK) keep[q] = 0;
  __syncthreads();
  // (eight earlier clauses are read before any is tested, so the reads of
  // one step overlap instead of each waiting for the last)
  auto strict_subset = [](const rp_clause& b, const rp_clause& a) {
    return (b.pos & ~a.pos) == 0 && (b.neg & ~a.neg) == 0 && (b.pos != a.pos || b.neg != a.neg);
  };
  for (uint32_t a = tid; a < n; a += CL_BLOCK) {
    const rp_clause ca = sc[a];
    bool k = a == 0 || sc[a - 1].pos != ca.pos || sc[a - 1].neg != ca.neg;
    uint32_t b = 0;
    for (; k && b + 8 <= a; b += 8) {
      rp_clause cb[8];
#pragma unroll
      for (int u = 0; u < 8; u++) cb[u] = sc[b + u];
#pragma unroll
      for (int u = 0; u < 8; u++)
        if (strict_subset(cb[u], ca)) k = false;
    }
    for (; k && b < a; b++)
      if (strict_subset(sc[b], ca)) k = false;
    if (k) atomicOr(&keep[a >> 5], 1u << (a & 31));
  }
  __syncthreads();
  // compaction in order: thread t owns clauses [t*per, (t+1)*per)
  const uint32_t per = (n + CL_BLOCK - 1) / CL_BLOCK;
  uint32_t mine = 0;
  for (uint32_t q = 0; q < per; q++) {
    const uint32_t a = tid * per + q;
    if (a < n && ((keep[a >> 5] >> (a & 31)) & 1)) mine++;
  }
  uint32_t total;
  uint32_t pos = block_excl_scan1024(mine, sm, &total);
  if (total > J.phi_cap) {
    if (tid == 0) { st->err = ERR_PHI_CAP; st->state = ST_ERROR; }
    return;
  }
  for (uint32_t q = 0; q < per; q++) {
    const uint32_t a = tid * per + q;
    if (a < n && ((keep[a >> 5] >> (a & 31)) & 1)) J.phi[pos++] = sc[a];
  }
  if (tid == 0) st->n_phi = total;
}

// Number of jobs still running, for the host's per-round check (4 bytes).
__global__ __launch_bounds__(256) void count_active_kernel(const Job* __restrict__ jobs,
                                                           uint32_t njobs, uint32_t* out) {
  __shared__ uint32_t s_n;
  if (threadIdx.x == 0) s_n = 0;
  __syncthreads();
  uint32_t c = 0;
  for (uint32_t j = threadIdx.x; j < njobs; j += 256) c += jobs[j].st->state == ST_RUN;
  if (c) atomicAdd(&s_n, c);
  __syncthreads();
  if (threadIdx.x == 0) *out = s_n;
}

hipError_t launch_count_active(const Job* jobs, uint32_t njobs, uint32_t* out, hipStream_t s) {
  count_active_kernel<<<1, 256, 0, s>>>(jobs, njobs, out);
  return hipGetLastError();
}

hipError_t launch_clause(const Job* jobs, uint32_t njobs, int learn, hipStream_t s) {
  if (njobs == 0) return hipSuccess;
  clause_kernel<<<njobs, CL_BLOCK, 0, s>>>(jobs, learn);
  return hipGetLastError();
}

}  // namespace rp

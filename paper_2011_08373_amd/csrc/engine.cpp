// Execution engine: lays out one or many jobs in a device workspace and runs
// record generation, the radix sort and the per-round Verify / GenerateClause /
// Solve kernels of Alg. 1 on a stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <vector>

#include "common.h"
#include "launch.h"
#include "plan.h"

namespace rp {

namespace {

constexpr size_t ALIGN = 256;
size_t up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

struct Layout {
  size_t total = 0, meta = 0;
  size_t o_jobs = 0, o_states = 0, o_items = 0, o_ssegs = 0, o_csegs = 0;
  size_t o_phi0 = 0;
  std::vector<size_t> o_pts, o_bany, o_bgrid, o_w, o_cpre, o_gpre, o_phi0j, o_wbits;
  size_t o_chunks = 0;
  size_t o_recA = 0, o_recB = 0, o_dig = 0, o_cnt = 0, o_tot = 0, o_off = 0, o_err = 0;
  std::vector<size_t> o_ivl, o_minj, o_j0, o_phi, o_scratch, o_traj, o_bitmap, o_pairs, o_ptotal;
  std::vector<uint32_t> phi_cap, scratch_cap;
  uint64_t n_rec = 0;
  uint32_t rb = 8, passes = 0;   // widest digit of the passes (table sizes), passes
  std::vector<DigitPass> digits;  // the passes' digits in execution order
  uint32_t n_chunks = 0;          // sort chunks = generation items (built on the device)
  uint32_t n_cblk = 0, max_cblk = 0;   // column blocks, and the most of one segment
  size_t o_part = 0;              // per column block and digit: its count, then its base
  uint64_t chunk_len = 0;
  std::vector<SortSeg> ssegs;
  std::vector<uint32_t> seg_job, seg_level;
};

uint32_t pow2_at_least(uint64_t n) {
  uint32_t p = 1;
  while (p < n) p <<= 1;
  return p;
}

void plan_layout(const std::vector<JobInput>& jobs, const EngineOpts& o, Layout& L) {
  const size_t N = jobs.size();
  // records and sort segments (two logs per job)
  uint32_t key_bits = 0;
  for (const JobInput& j : jobs) key_bits = std::max(key_bits, j.plan->key_bits);
  L.digits = digit_plan(key_bits);
  L.passes = (uint32_t)L.digits.size();
  L.rb = 6;
  for (const DigitPass& dp : L.digits) L.rb = std::max(L.rb, dp.bits);
  uint64_t rec = 0;
  for (size_t j = 0; j < N; j++) {
    const Plan& p = *jobs[j].plan;
    for (int v = 0; v < 2; v++) {
      const uint64_t n = v == 0 ? p.n_intra : p.n_inter;
      if (n == 0) continue;
      SortSeg s{};
      s.beg = rec;
      s.end = rec + n;
      s.shift = p.key_shift;
      s.job = (uint32_t)j;
      s.view = (uint32_t)v;
      L.ssegs.push_back(s);
      L.seg_job.push_back((uint32_t)j);
      L.seg_level.push_back((uint32_t)v);
      rec += n;
    }
  }
  L.n_rec = rec;
  // sort chunks (= generation items): whole sort tiles, at most ~16K chunks
  // (the per-chunk digit counts and offsets of each pass are read and
  // written by the column scans: fewer, longer chunks keep those tables
  // small on billion-record logs)
  const uint64_t tile = sort_tile_size();
  uint64_t chunk = std::max<uint64_t>(2 * tile, (rec + 16383) / 16384);
  chunk = (chunk + tile - 1) / tile * tile;
  L.chunk_len = chunk;
  for (size_t s = 0; s < L.ssegs.size(); s++) {
    L.ssegs[s].chunk_beg = L.n_chunks;
    L.n_chunks += (uint32_t)((L.ssegs[s].end - L.ssegs[s].beg + chunk - 1) / chunk);
    L.ssegs[s].chunk_end = L.n_chunks;
    const uint32_t nb = (L.ssegs[s].chunk_end - L.ssegs[s].chunk_beg + COL_BLOCK_CHUNKS - 1) /
                        COL_BLOCK_CHUNKS;
    L.ssegs[s].cblk_beg = L.n_cblk;
    L.n_cblk += nb;
    L.max_cblk = std::max(L.max_cblk, nb);
  }
  const uint32_t R = 1u << L.rb;
  // ---- meta region (uploaded)
  size_t off = 0;
  L.o_jobs = off; off = up(off + N * sizeof(Job));
  L.o_states = off; off = up(off + N * sizeof(JobState));
  // words: 0 error, 8 running-job count, 9 conflict-tile counter, 10 scatter
  // chunk ticket; uploaded as zeros
  L.o_err = off; off = up(off + 64);
  L.o_ssegs = off; off = up(off + L.ssegs.size() * sizeof(SortSeg));
  L.o_csegs = off; off = up(off + L.ssegs.size() * sizeof(ConfSeg));
  L.o_pts.resize(N); L.o_bany.resize(N); L.o_bgrid.resize(N); L.o_w.resize(N);
  L.o_wbits.resize(N);
  L.o_cpre.resize(N); L.o_gpre.resize(N); L.o_phi0j.resize(N);
  for (size_t j = 0; j < N; j++) {
    const Plan& p = *jobs[j].plan;
    L.o_pts[j] = off; off = up(off + p.P * sizeof(DPoint));
    L.o_wbits[j] = off; off = up(off + p.wbits.size() * sizeof(uint64_t));
    L.o_bany[j] = off; off = up(off + p.P * sizeof(uint64_t));
    L.o_bgrid[j] = off; off = up(off + p.P * sizeof(uint64_t));
    L.o_w[j] = off; off = up(off + p.S * sizeof(uint32_t));
    L.o_cpre[j] = off; off = up(off + (p.P + 1) * sizeof(uint64_t));
    L.o_gpre[j] = off; off = up(off + (p.P + 1) * sizeof(uint64_t));
    L.o_phi0j[j] = off; off = up(off + jobs[j].phi0.size() * sizeof(rp_clause));
  }
  L.meta = off;
  // ---- device-only region
  L.o_items = off; off = up(off + (size_t)L.n_chunks * sizeof(GenItem));
  L.o_chunks = off; off = up(off + (size_t)L.n_chunks * sizeof(SortChunk));
  L.o_recA = off; off = up(off + L.n_rec * sizeof(uint64_t));
  L.o_recB = off; off = up(off + L.n_rec * sizeof(uint64_t));   // sort ping-pong, then run log
  // each record's digit of the next pass, written by a scatter beside its
  // output and counted by the next pass (read as whole 16-byte vectors)
  if (L.passes > 1) {
    uint32_t wide = 1;            // bytes per stored digit: 2 if any pass after the first has
    for (uint32_t p = 1; p < L.passes; p++)    // more than 8 bits
      if (L.digits[p].bits > 8) wide = 2;
    L.o_dig = off;
    off = up(off + L.n_rec * wide + 16);
  }
  L.o_cnt = off; off = up(off + (size_t)L.n_chunks * R * sizeof(uint32_t));
  L.o_tot = off; off = up(off + L.ssegs.size() * (size_t)R * sizeof(uint64_t));
  L.o_part = off; off = up(off + (size_t)L.n_cblk * R * sizeof(uint64_t));
  L.o_off = off; off = up(off + (size_t)L.n_chunks * R * sizeof(uint64_t));
  L.o_ivl.resize(N); L.o_minj.resize(N); L.o_j0.resize(N); L.o_phi.resize(N); L.o_scratch.resize(N);
  L.o_traj.resize(N); L.o_bitmap.resize(N); L.o_pairs.resize(N); L.o_ptotal.resize(N);
  L.phi_cap.resize(N); L.scratch_cap.resize(N);
  for (size_t j = 0; j < N; j++) {
    const Plan& p = *jobs[j].plan;
    // reduced phi holds at most one race clause per (point, level), one
    // divergence unit per slot and the option units
    const uint32_t cap = 2 * p.P + 2 * 64 + 64 + (uint32_t)jobs[j].phi0.size();
    L.phi_cap[j] = cap;
    L.scratch_cap[j] = pow2_at_least((uint64_t)cap + 2 * p.P + 64);
    L.o_ivl[j] = off; off = up(off + 2 * p.P * sizeof(uint32_t));
    L.o_minj[j] = off; off = up(off + 2 * p.P * sizeof(uint32_t));
    L.o_j0[j] = off; off = up(off + 2 * p.P * sizeof(uint32_t));
    L.o_phi[j] = off; off = up(off + L.phi_cap[j] * sizeof(rp_clause));
    L.o_scratch[j] = off; off = up(off + L.scratch_cap[j] * sizeof(rp_clause));
    L.o_traj[j] = off; off = up(off + o.traj_cap * sizeof(uint64_t));
    if (o.op == OP_CHECK) {
      const uint64_t wpr = (p.P + 63) / 64;
      L.o_bitmap[j] = off; off = up(off + 2 * (uint64_t)p.P * wpr * sizeof(uint64_t));
      L.o_pairs[j] = off; off = up(off + (uint64_t)p.P * (p.P + 1) * sizeof(rp_pair));
      L.o_ptotal[j] = off; off = up(off + sizeof(uint64_t));
    }
  }
  L.total = off;
}

// Phase timing with hipEvents from a per-thread, per-device pool: creating
// events costs host time on every call, so they are made once and reused.
// A timer takes the pool entries above the ones held by timers still alive
// on the thread, and hands them back when it ends (after the call has
// synchronised its stream).
struct EventPool {
  std::map<int, std::vector<hipEvent_t>> ev;   // by device
  std::map<int, size_t> top;
};
static thread_local EventPool t_pool;

// A mark records an event when the timer's level reaches the mark's level
// (1: the streaming kernels and the total, 2: every phase).
struct Timer {
  std::vector<hipEvent_t> ev;
  std::vector<int> tag;
  hipStream_t s;
  bool ok = true;
  bool on = true;
  int level = 0;
  int dev = 0;
  size_t base = 0;
  explicit Timer(hipStream_t st, int lvl) : s(st), on(lvl > 0), level(lvl) {
    if (on && hipGetDevice(&dev) != hipSuccess) on = false;
    if (on) base = t_pool.top[dev];
  }
  void mark(int t, int min_level = 1) {
    if (!on || level < min_level) return;
    std::vector<hipEvent_t>& pool = t_pool.ev[dev];
    size_t& top = t_pool.top[dev];
    if (top == pool.size()) {
      // timing only: no system-scope fence when the event is recorded (no
      // cache write-back and invalidation between the timed kernels); the
      // call synchronises its stream before it reads the times
      hipEvent_t e;
      if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
        ok = false;
        return;
      }
      pool.push_back(e);
    }
    hipEvent_t e = pool[top++];
    if (hipEventRecord(e, s) != hipSuccess) ok = false;
    ev.push_back(e);
    tag.push_back(t);
  }
  ~Timer() {
    if (on) t_pool.top[dev] = base;
  }
};

// phase tags for the stats
// T_ROUND opens a repair round: the time since the previous mark (the
// host's per-round readback) is counted in ms_total only.
enum { T_START = 0, T_UPLOAD, T_GEN, T_SORTPASS, T_SORT, T_RUNS, T_SUMPRE, T_SUMMARY, T_ROUND,
       T_CONFPRE, T_CHECK, T_CLAUSE, T_SOLVE, T_END };

}  // namespace

size_t engine_workspace(const std::vector<JobInput>& jobs, const EngineOpts& o) {
  Layout L;
  plan_layout(jobs, o, L);
  return L.total;
}

#define HIPCHK(x)                          \
  do {                                     \
    if ((x) != hipSuccess) return RP_ERR_DEVICE; \
  } while (0)

// Page-locked host staging for the descriptor upload, one per host thread,
// grown on demand and kept for the life of the thread (never freed: a
// thread-exit free could run after the runtime is gone).  An event marks the
// last upload out of it; the next call waits for that event before writing.
struct PinnedStage {
  uint8_t* p = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
  bool pending = false;
  uint8_t* get(size_t n) {
    if (pending) {
      if (!done || hipEventSynchronize(done) != hipSuccess) return nullptr;
      pending = false;
    }
    if (n > cap) {
      if (p) (void)hipHostFree(p);
      p = nullptr;
      cap = 0;
      if (hipHostMalloc((void**)&p, n < 4096 ? 4096 : n, hipHostMallocDefault) != hipSuccess) {
        p = nullptr;
        return nullptr;
      }
      cap = n < 4096 ? 4096 : n;
    }
    return p;
  }
  // page-locked space for results read back by this thread's calls (each
  // call waits for its copies before it returns)
  uint8_t* rb = nullptr;
  size_t rb_cap = 0;
  template <class T = uint32_t>
  T* readback(size_t n) {
    if (n > rb_cap) {
      if (rb) (void)hipHostFree(rb);
      rb = nullptr;
      rb_cap = 0;
      const size_t want = n < 4096 ? 4096 : n;
      if (hipHostMalloc((void**)&rb, want, hipHostMallocDefault) != hipSuccess) {
        rb = nullptr;
        return nullptr;
      }
      rb_cap = want;
    }
    return reinterpret_cast<T*>(rb);
  }
  // the uploads out of the buffer were enqueued on s
  void in_flight(hipStream_t s) {
    if (!done && hipEventCreateWithFlags(&done, hipEventDisableTiming) != hipSuccess) done = nullptr;
    if (done && hipEventRecord(done, s) == hipSuccess) pending = true;
    else (void)hipStreamSynchronize(s);
  }
};
thread_local PinnedStage t_stage;

namespace {

// Host staging (hbuf, L.meta bytes, must stay untouched until the upload
// enqueued here has run), upload, record generation, sort and first-partner
// table for the jobs laid out by L in the device buffer d (all enqueued on
// s, no sync).
int prepare_jobs(const std::vector<JobInput>& jobs, const EngineOpts& o, const Layout& L,
                 uint8_t* d, uint8_t* hbuf, hipStream_t s, Timer& tm) {
  const size_t N = jobs.size();
  // the job and state tables and the error words come first and are the
  // only ones not written in full below
  std::memset(hbuf, 0, L.o_ssegs);
  Job* hj = (Job*)(hbuf + L.o_jobs);
  JobState* hs = (JobState*)(hbuf + L.o_states);
  for (size_t j = 0; j < N; j++) {
    const Plan& p = *jobs[j].plan;
    Job& J = hj[j];
    J.P = p.P; J.S = p.S; J.B = p.B; J.T = p.T;
    J.tbits = p.tbits; J.bbits = p.bbits; J.pbits = p.pbits; J.key_shift = p.key_shift;
    J.nbits = p.nbits; J.policy = jobs[j].policy;
    J.pts = (const DPoint*)(d + L.o_pts[j]);
    J.wbits = (const uint64_t*)(d + L.o_wbits[j]);
    J.bits_any = (const uint64_t*)(d + L.o_bany[j]);
    J.bits_grid = (const uint64_t*)(d + L.o_bgrid[j]);
    J.weights = (const uint32_t*)(d + L.o_w[j]);
    J.cnt_pre = (const uint64_t*)(d + L.o_cpre[j]);
    J.gcnt_pre = (const uint64_t*)(d + L.o_gpre[j]);
    J.rblk = p.cnt_pre.empty() ? 0 : p.cnt_pre[p.P];
    J.div_if_enabled = p.div_if_enabled;
    J.pad_array = p.pad_array;
    J.log[0] = J.log[1] = nullptr;
    J.nlog[0] = p.n_intra;
    J.nlog[1] = p.n_inter;
    J.ivl = (uint32_t*)(d + L.o_ivl[j]);
    J.minj = (uint32_t*)(d + L.o_minj[j]);
    J.j0 = (uint32_t*)(d + L.o_j0[j]);
    J.bitmap = o.op == OP_CHECK ? (uint64_t*)(d + L.o_bitmap[j]) : nullptr;
    J.wpr = (p.P + 63) / 64;
    J.phi = (rp_clause*)(d + L.o_phi[j]);
    J.scratch = (rp_clause*)(d + L.o_scratch[j]);
    J.phi_cap = L.phi_cap[j];
    J.scratch_cap = L.scratch_cap[j];
    J.st = (JobState*)(d + L.o_states) + j;
    J.traj = o.traj_cap ? (uint64_t*)(d + L.o_traj[j]) : nullptr;
    J.traj_cap = o.traj_cap;
    J.node_limit = 1ull << solver_nodes_log2(0, false);
    JobState& S = hs[j];
    std::memset(&S, 0, sizeof(S));
    S.x = jobs[j].x;
    S.n_phi = (uint32_t)jobs[j].phi0.size();
    S.state = ST_RUN;
    S.max_rounds = jobs[j].max_rounds;
    S.phase = jobs[j].solver ? PH_GREEDY : PH_EXACT;
    std::memcpy(hbuf + L.o_pts[j], p.pts.data(), p.P * sizeof(DPoint));
    std::memcpy(hbuf + L.o_wbits[j], p.wbits.data(), p.wbits.size() * sizeof(uint64_t));
    std::memcpy(hbuf + L.o_bany[j], p.bits_any.data(), p.P * sizeof(uint64_t));
    std::memcpy(hbuf + L.o_bgrid[j], p.bits_grid.data(), p.P * sizeof(uint64_t));
    std::memcpy(hbuf + L.o_w[j], p.weights.data(), p.S * sizeof(uint32_t));
    std::memcpy(hbuf + L.o_cpre[j], p.cnt_pre.data(), (p.P + 1) * sizeof(uint64_t));
    std::memcpy(hbuf + L.o_gpre[j], p.gcnt_pre.data(), (p.P + 1) * sizeof(uint64_t));
    std::memcpy(hbuf + L.o_phi0j[j], jobs[j].phi0.data(), jobs[j].phi0.size() * sizeof(rp_clause));
  }
  std::memcpy(hbuf + L.o_ssegs, L.ssegs.data(), L.ssegs.size() * sizeof(SortSeg));
  // sorted logs end in buffer A after an even number of passes, else B
  uint8_t* sorted = d + ((L.passes % 2 == 0) ? L.o_recA : L.o_recB);
  ConfSeg* hc = (ConfSeg*)(hbuf + L.o_csegs);
  for (size_t q = 0; q < L.ssegs.size(); q++) {
    ConfSeg c{};
    c.log = (const uint64_t*)sorted + L.ssegs[q].beg;
    c.n = L.ssegs[q].end - L.ssegs[q].beg;
    c.job = L.seg_job[q];
    c.level = L.seg_level[q];
    c.ctile_beg = 0;     // laid out on the device before each scan
    hc[q] = c;
    hj[c.job].log[c.level] = c.log;
  }
  tm.mark(T_START);
  HIPCHK(hipMemcpyAsync(d, hbuf, L.meta, hipMemcpyHostToDevice, s));
  for (size_t j = 0; j < N; j++)
    if (!jobs[j].phi0.empty())
      HIPCHK(hipMemcpyAsync(d + L.o_phi[j], d + L.o_phi0j[j],
                            jobs[j].phi0.size() * sizeof(rp_clause), hipMemcpyDeviceToDevice, s));
  HIPCHK(launch_items((const Job*)(d + L.o_jobs), (const SortSeg*)(d + L.o_ssegs),
                      (uint32_t)L.ssegs.size(), L.n_chunks, L.chunk_len, (GenItem*)(d + L.o_items),
                      (SortChunk*)(d + L.o_chunks), s));
  tm.mark(T_UPLOAD);
  const Job* djobs = (const Job*)(d + L.o_jobs);
  uint32_t* derr = (uint32_t*)(d + L.o_err);
  // ---- records and sort
  const int passes = (int)L.passes;
  const SortSeg* dss = (const SortSeg*)(d + L.o_ssegs);
  const SortChunk* dch = (const SortChunk*)(d + L.o_chunks);
  const uint32_t nch = L.n_chunks;
  uint32_t* dcnt = (uint32_t*)(d + L.o_cnt);
  uint64_t* dtot = (uint64_t*)(d + L.o_tot);
  uint64_t* doff = (uint64_t*)(d + L.o_off);
  // each pass's digit (digit_plan: any fixed order of the digits leaves
  // every location's records together and in generation order, and the
  // scans need nothing more); generation counts the first pass's digit
  const std::vector<DigitPass>& dg = L.digits;
  HIPCHK(launch_gen(passes > 0 ? (int)dg[0].bits : 8, (const GenItem*)(d + L.o_items), nch,
                    djobs, dss, (uint64_t*)(d + L.o_recA), dcnt,
                    passes > 0 ? (int)dg[0].lo : -1, s));
  tm.mark(T_GEN);
  for (int p = 0; p < passes; p++) {
    const uint64_t* in = (const uint64_t*)(d + ((p % 2 == 0) ? L.o_recA : L.o_recB));
    uint64_t* out = (uint64_t*)(d + ((p % 2 == 0) ? L.o_recB : L.o_recA));
    void* dig = L.passes > 1 ? (void*)(d + L.o_dig) : nullptr;
    const bool last = p + 1 == passes;
    HIPCHK(launch_sort_scan((int)dg[p].bits, dig, dss, (uint32_t)L.ssegs.size(), dch, nch,
                            L.n_cblk, L.max_cblk, dcnt, dtot, (uint64_t*)(d + L.o_part), doff,
                            derr + 10, p == 0, s));
    tm.mark(T_SORTPASS);
    HIPCHK(launch_sort_scatter((int)dg[p].bits, p, in, out, dss, dch, nch, (int)dg[p].lo,
                               last ? 0 : (int)dg[p + 1].lo, last ? 0 : (int)dg[p + 1].bits,
                               doff, derr + 10, derr, last ? nullptr : dig, s));
    tm.mark(T_SORT);
  }
  tm.mark(T_SORT, 2);
  ConfSeg* dcs = (ConfSeg*)(d + L.o_csegs);
  // ---- first partners with no barrier enabled (once per job): every
  // later Verify call resolves its first partners from them
  // (a job without access records keeps the cleared table: no partner)
  if (o.op != OP_CHECK && o.op != OP_SOLVE) {
    uint32_t maxP = 1;
    bool lo32 = true;
    for (const JobInput& j : jobs) {
      maxP = std::max(maxP, j.plan->P);
      lo32 = lo32 && j.plan->tbits < 32 && j.plan->bbits < 32 &&
             j.plan->tbits + j.plan->bbits + j.plan->pbits <= 32;
    }
    HIPCHK(launch_ivl(djobs, (uint32_t)N, IVL_ZERO, s));
    if (!L.ssegs.empty()) {
      HIPCHK(launch_conf_tiles(djobs, dcs, (int)L.ssegs.size(), derr + 9, s));
      tm.mark(T_SUMPRE);
      HIPCHK(launch_j0(djobs, dcs, (int)L.ssegs.size(), maxP, lo32, derr + 9, s));
      tm.mark(T_SUMMARY);
    }
    HIPCHK(launch_save_j0(djobs, (uint32_t)N, s));
  }
  return RP_OK;
}

}  // namespace

size_t engine_job_bytes(const JobInput& job) {
  std::vector<JobInput> v{job};
  return engine_group_bytes(v);
}

size_t engine_group_bytes(const std::vector<JobInput>& jobs) {
  EngineOpts o;
  o.op = OP_REPAIR;
  return engine_workspace(jobs, o);
}

int engine_prepare_group(const std::vector<JobInput>& jobs, void* region, size_t bytes,
                         hipStream_t s, std::vector<PreparedJob>& out,
                         std::vector<uint8_t>& staging) {
  EngineOpts o;
  o.op = OP_REPAIR;
  Layout L;
  plan_layout(jobs, o, L);
  if (bytes < L.total || !region) return RP_ERR_WORKSPACE;
  uint8_t* d = (uint8_t*)region;
  Timer tm(s, 0);
  staging.resize(L.meta);
  const int rc = prepare_jobs(jobs, o, L, d, staging.data(), s, tm);
  if (rc != RP_OK) return rc;
  // the first Solve of the jobs with option units (an empty phi is
  // answered by the initial x = 0): over the whole group, the others are
  // left as they are by the solver
  bool any_units = false;
  for (const JobInput& j : jobs) any_units |= !j.phi0.empty();
  if (any_units) HIPCHK(launch_solve((const Job*)(d + L.o_jobs), (uint32_t)jobs.size(), s));
  out.resize(jobs.size());
  for (size_t j = 0; j < jobs.size(); j++)
    std::memcpy(&out[j].job, staging.data() + L.o_jobs + j * sizeof(Job), sizeof(Job));
  return RP_OK;
}

int engine_round(const Job* djobs, uint32_t njobs, uint32_t* dactive, hipStream_t s) {
  HIPCHK(launch_ivl(djobs, njobs, IVL_RESOLVE, s));
  HIPCHK(launch_clause(djobs, njobs, 1, s));
  HIPCHK(launch_solve(djobs, njobs, s));
  HIPCHK(launch_count_active(djobs, njobs, dactive, s));
  return RP_OK;
}

int engine_run(const std::vector<JobInput>& jobs, const EngineOpts& o, void* ws, size_t ws_bytes,
               hipStream_t s, std::vector<JobResult>& res, rp_stats* stats) {
  Layout L;
  plan_layout(jobs, o, L);
  if (ws_bytes < L.total) return RP_ERR_WORKSPACE;
  if (!ws && L.total) return RP_ERR_WORKSPACE;
  const size_t N = jobs.size();
  uint8_t* d = (uint8_t*)ws;
  Timer tm(s, o.no_alloc ? 0 : timing_level(0, false));
  // host staging: page-locked and kept per thread, or (no_alloc) ordinary
  // memory, which the upload has read before hipMemcpyAsync returns
  static thread_local std::vector<uint8_t> plain_stage, plain_rb;
  if (o.no_alloc) {
    plain_stage.resize(L.meta);
    const int rc = prepare_jobs(jobs, o, L, d, plain_stage.data(), s, tm);
    if (rc != RP_OK) return rc;
  } else {
    uint8_t* h = t_stage.get(L.meta);
    if (!h) return RP_ERR_DEVICE;
    const int rc = prepare_jobs(jobs, o, L, d, h, s, tm);
    t_stage.in_flight(s);
    if (rc != RP_OK) return rc;
  }
  const Job* djobs = (const Job*)(d + L.o_jobs);
  uint32_t* derr = (uint32_t*)(d + L.o_err);
  ConfSeg* dcs = (ConfSeg*)(d + L.o_csegs);
  tm.mark(T_RUNS, 2);
  // ---- per-round kernels
  const int nseg = (int)L.ssegs.size();
  uint32_t* dtiles = derr + 9;     // conf tiles of the all-pairs scan
  uint32_t maxP = 1;
  for (const JobInput& j : jobs) maxP = std::max(maxP, j.plan->P);
  std::vector<JobState> hst(N);
  // job states, the error word and the start of each job's trajectory (the
  // usual few rounds) are read back into page-locked memory in one go
  const uint32_t traj_head = std::min<uint32_t>(o.traj_cap, 16);
  const size_t rb_bytes = N * sizeof(JobState) + 64 + N * traj_head * sizeof(uint64_t);
  uint8_t* rb;
  if (o.no_alloc) {
    plain_rb.resize(rb_bytes);
    rb = plain_rb.data();
  } else {
    rb = (uint8_t*)t_stage.readback(rb_bytes);
  }
  if (!rb) return RP_ERR_DEVICE;
  JobState* pst = (JobState*)rb;
  uint32_t* herr = (uint32_t*)(rb + N * sizeof(JobState));
  uint64_t* ptraj = (uint64_t*)(rb + N * sizeof(JobState) + 64);
  auto enqueue_results = [&]() -> hipError_t {
    hipError_t e = hipMemcpyAsync(pst, d + L.o_states, N * sizeof(JobState), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(herr, derr, 64, hipMemcpyDeviceToHost, s);
    for (size_t j = 0; j < N && traj_head && e == hipSuccess; j++)
      e = hipMemcpyAsync(ptraj + j * traj_head, d + L.o_traj[j], traj_head * sizeof(uint64_t),
                         hipMemcpyDeviceToHost, s);
    return e;
  };
  bool ended = false, have_results = false;
  // the run logs are scanned once: by the all-pairs scan of a check, else
  // by the first-partner scan of the preparation
  const uint64_t scanned = o.op == OP_SOLVE ? 0 : L.n_rec;
  uint32_t rounds_run = 0;
  const uint32_t conf_launches = o.op == OP_SOLVE ? 0 : 1;
  if (o.op == OP_CHECK) {
    HIPCHK(launch_ivl(djobs, (uint32_t)N, IVL_CHECK, s));
    HIPCHK(launch_conf_tiles(djobs, dcs, nseg, dtiles, s));
    tm.mark(T_CONFPRE);
    HIPCHK(launch_conf(djobs, dcs, nseg, maxP, dtiles, s));
    tm.mark(T_CHECK);
    for (size_t j = 0; j < N; j++)
      HIPCHK(launch_pairs(djobs + j, (rp_pair*)(d + L.o_pairs[j]), (uint64_t*)(d + L.o_ptotal[j]), s));
    tm.mark(T_CLAUSE);
  } else if (o.op == OP_SOLVE) {
    HIPCHK(launch_solve(djobs, (uint32_t)N, s));
    tm.mark(T_SOLVE);
  } else if (o.op == OP_FIRST) {
    HIPCHK(launch_ivl(djobs, (uint32_t)N, IVL_RESOLVE, s));
    tm.mark(T_CHECK);
  } else if (o.op == OP_CLAUSES) {
    HIPCHK(launch_ivl(djobs, (uint32_t)N, IVL_RESOLVE, s));
    tm.mark(T_CHECK);
    HIPCHK(launch_clause(djobs, (uint32_t)N, 1, s));
    tm.mark(T_CLAUSE);
  } else {
    uint32_t* dactive = (uint32_t*)(d + L.o_err) + 8;
    // the first Solve of Alg. 1: with no option units phi is empty and its
    // answer is x = 0 (weight 0), which the job states already hold
    bool any_units = false;
    for (const JobInput& j : jobs) any_units |= !j.phi0.empty();
    if (any_units) HIPCHK(launch_solve(djobs, (uint32_t)N, s));
    tm.mark(T_SOLVE, 2);
    auto round = [&]() -> hipError_t {
      hipError_t e;
      if ((e = launch_ivl(djobs, (uint32_t)N, IVL_RESOLVE, s)) != hipSuccess) return e;
      if ((e = launch_clause(djobs, (uint32_t)N, 1, s)) != hipSuccess) return e;
      if ((e = launch_solve(djobs, (uint32_t)N, s)) != hipSuccess) return e;
      return launch_count_active(djobs, (uint32_t)N, dactive, s);
    };
    // the first round is launched directly; if jobs remain, the round is
    // captured once in a graph and replayed until every job has a verdict.
    // A small batch reads every verdict together with the round's count of
    // running jobs (it sits in the error word), so the round that ends the
    // loop needs no further wait; a large one reads the count alone.
    const bool with_results = N <= 64;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    bool tried_graph = false;
    uint32_t n_active = 1;
    int rc_loop = RP_OK;
    while (n_active) {
      if (rounds_run == 1 && !tried_graph && o.use_graph && s != nullptr) {
        tried_graph = true;
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess) {
          const hipError_t e = round();
          const hipError_t ec = hipStreamEndCapture(s, &graph);
          if (e != hipSuccess || ec != hipSuccess ||
              hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0) != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            graph = nullptr;
            gexec = nullptr;
            (void)hipGetLastError();
          }
        }
      }
      tm.mark(T_ROUND, 2);
      if (gexec) {
        if (hipGraphLaunch(gexec, s) != hipSuccess) { rc_loop = RP_ERR_DEVICE; break; }
        tm.mark(T_CHECK, 2);
      } else {
        HIPCHK(launch_ivl(djobs, (uint32_t)N, IVL_RESOLVE, s));
        tm.mark(T_CHECK, 2);
        HIPCHK(launch_clause(djobs, (uint32_t)N, 1, s));
        tm.mark(T_CLAUSE, 2);
        HIPCHK(launch_solve(djobs, (uint32_t)N, s));
        tm.mark(T_SOLVE, 2);
        HIPCHK(launch_count_active(djobs, (uint32_t)N, dactive, s));
      }
      tm.mark(T_END);           // the last one recorded ends the final round
      const hipError_t e = with_results
                               ? enqueue_results()
                               : hipMemcpyAsync(herr + 8, dactive, sizeof(uint32_t),
                                                hipMemcpyDeviceToHost, s);
      if (e != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
        rc_loop = RP_ERR_DEVICE;
        break;
      }
      n_active = herr[8];
      rounds_run++;
      if (rounds_run > 100000) { rc_loop = RP_ERR_DEVICE; break; }
    }
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (rc_loop != RP_OK) return rc_loop;
    ended = true;
    have_results = with_results;
  }
  if (!ended) tm.mark(T_END);
  if (!have_results) {
    HIPCHK(enqueue_results());
    HIPCHK(hipStreamSynchronize(s));
  }
  std::memcpy(hst.data(), pst, N * sizeof(JobState));
  if (herr[0]) return RP_ERR_DEVICE;
  res.assign(N, JobResult{});
  for (size_t j = 0; j < N; j++) {
    res[j].st = hst[j];
    // a job that failed on the device keeps its own error state; the other
    // jobs of the call are unaffected and read out as usual
    if (hst[j].state == ST_ERROR) continue;
    if (o.op == OP_FIRST) {
      res[j].first.resize(2 * (size_t)jobs[j].plan->P);
      if (!res[j].first.empty())
        HIPCHK(hipMemcpyAsync(res[j].first.data(), d + L.o_minj[j],
                              res[j].first.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    }
    if (o.op == OP_CLAUSES) {
      res[j].phi.resize(hst[j].n_phi);
      if (hst[j].n_phi)
        HIPCHK(hipMemcpyAsync(res[j].phi.data(), d + L.o_phi[j], hst[j].n_phi * sizeof(rp_clause),
                              hipMemcpyDeviceToHost, s));
    }
    if (o.op == OP_CHECK) {
      uint64_t tot = 0;
      HIPCHK(hipMemcpyAsync(&tot, d + L.o_ptotal[j], sizeof(tot), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      res[j].n_pairs = tot;
      if (o.want_pairs && tot <= o.pair_cap && tot) {
        res[j].pairs.resize(tot);
        HIPCHK(hipMemcpyAsync(res[j].pairs.data(), d + L.o_pairs[j], tot * sizeof(rp_pair),
                              hipMemcpyDeviceToHost, s));
      }
    }
    if (o.traj_cap) {
      const uint32_t nt = std::min(hst[j].rounds, o.traj_cap);
      res[j].traj.resize(nt);
      if (nt <= traj_head)
        std::memcpy(res[j].traj.data(), ptraj + j * traj_head, nt * sizeof(uint64_t));
      else
        HIPCHK(hipMemcpyAsync(res[j].traj.data(), d + L.o_traj[j], nt * sizeof(uint64_t),
                              hipMemcpyDeviceToHost, s));
    }
  }
  HIPCHK(hipStreamSynchronize(s));
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    for (size_t q = 1; q < tm.ev.size(); q++) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, tm.ev[q - 1], tm.ev[q]) != hipSuccess) continue;
      switch (tm.tag[q]) {
        case T_GEN: stats->ms_gen += ms; break;
        case T_SORTPASS: stats->ms_sort += ms; break;
        case T_SORT:
          stats->ms_sort += ms;
          if (tm.tag[q - 1] == T_SORTPASS) {
            stats->ms_sort_kernels += ms;
            stats->ms_sort_pass_max = std::max(stats->ms_sort_pass_max, (double)ms);
            stats->sort_launches++;
          }
          break;
        case T_UPLOAD: stats->ms_upload += ms; break;
        case T_RUNS: stats->ms_j0 += ms; break;
        case T_SUMPRE: stats->ms_j0 += ms; break;
        case T_SUMMARY:
          stats->ms_j0 += ms;
          stats->ms_conf_kernels += ms;
          break;
        case T_CONFPRE: stats->ms_check += ms; break;
        case T_CHECK:
          stats->ms_check += ms;
          if (tm.tag[q - 1] == T_CONFPRE) stats->ms_conf_kernels += ms;
          break;
        case T_CLAUSE: stats->ms_clause += ms; break;
        case T_SOLVE: stats->ms_solve += ms; break;
        default: break;
      }
    }
    float tot = 0;
    if (tm.ev.size() >= 2 && hipEventElapsedTime(&tot, tm.ev.front(), tm.ev.back()) == hipSuccess)
      stats->ms_total = tot;
    stats->records = L.n_rec;
    for (const JobInput& j : jobs) stats->accesses += j.plan->accesses;
    stats->records_scanned = scanned;
    stats->sort_passes = L.passes;
    stats->rounds = rounds_run;
    stats->conf_launches = conf_launches;
  }
  return RP_OK;
}

}  // namespace rp

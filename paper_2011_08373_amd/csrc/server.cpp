// Serving: continuous batching of repair jobs over a caller-owned device arena.
//
// Jobs are submitted at any time (the server copies their descriptors).  Each
// rp_server_step():
//   1. admits pending jobs in arrival order while they fit: the jobs
//      admitted in one step form a group that is laid out in one free range
//      of the arena (first fit) and prepared together, one launch per phase
//      for the whole group (upload, records, sort, run logs, first-partner
//      tables, first Solve) -- their logs and clause sets then stay resident,
//      and the range is released when the group's last job finishes;
//   2. runs one round of Alg. 1 (Verify, GenerateClause, Solve) over every
//      resident job at once, newly admitted ones included;
//   3. retires the jobs that reached a verdict, frees their ranges and
//      stamps their latency (submission to verdict).
// Each job's result is the one rp_repair gives for it alone: rounds only
// batch independent jobs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <vector>

#include "common.h"
#include "launch.h"
#include "plan.h"

namespace rp {

namespace {

constexpr size_t SALIGN = 256;
constexpr size_t MAX_GROUP = 256;   // jobs admitted (and prepared together) per step
size_t sup(size_t x) { return (x + SALIGN - 1) / SALIGN * SALIGN; }
double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct OwnedKernel {   // deep copy of a descriptor
  std::vector<rp_array> arrays;
  std::vector<rp_guard> guards, block_guards;
  std::vector<rp_point> points;
  std::vector<rp_slot> slots;
  rp_kernel k;
  void take(const rp_kernel* src) {
    arrays.assign(src->arrays, src->arrays + src->n_arrays);
    guards.assign(src->guards, src->guards + src->n_guards);
    if (src->block_guards)
      block_guards.assign(src->block_guards, src->block_guards + src->n_guards);
    else
      block_guards.clear();
    points.assign(src->points, src->points + src->n_points);
    slots.assign(src->slots, src->slots + src->n_slots);
    k = *src;
    k.arrays = arrays.data();
    k.guards = guards.data();
    k.block_guards = src->block_guards ? block_guards.data() : nullptr;
    k.points = points.data();
    k.slots = slots.data();
  }
};

struct SJob {
  uint64_t id = 0;
  OwnedKernel desc;
  Plan plan;
  JobInput input;
  size_t bytes = 0;            // footprint of the job prepared alone
  PreparedJob prep;
  double t_submit = 0;
  uint32_t group = 0;          // admission group holding its range
};

struct Group {
  size_t off = 0, bytes = 0;
  uint32_t live = 0;           // jobs of the group not yet finished
};

// first-fit allocator over [0, size)
struct Arena {
  std::map<size_t, size_t> free_;   // offset -> length
  void init(size_t base, size_t size) { free_.clear(); if (size) free_[base] = size; }
  bool alloc(size_t n, size_t& off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        off = it->first;
        const size_t rest = it->second - n;
        free_.erase(it);
        if (rest) free_[off + n] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

__global__ void gather_states_kernel(const Job* jobs, uint32_t n, JobState* out) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) out[j] = *jobs[j].st;
}

}  // namespace

struct Server {
  uint8_t* arena = nullptr;
  size_t arena_bytes = 0;
  rp_repair_opts opts{};
  hipStream_t s = nullptr;
  uint32_t max_resident = 0;
  // fixed tables at the start of the arena
  Job* d_jobs = nullptr;
  JobState* d_states = nullptr;
  uint32_t* d_active = nullptr;
  size_t tables = 0;
  Arena alloc;
  std::deque<std::unique_ptr<SJob>> pending;
  std::vector<std::unique_ptr<SJob>> resident;
  struct Done { uint64_t id; rp_repair_out out; double latency; };
  std::deque<Done> done;
  std::vector<uint8_t> staging;
  std::map<uint32_t, Group> groups;
  uint32_t next_group = 0;
  std::vector<Job> h_jobs;
  std::vector<JobState> h_states;
  uint64_t rounds = 0;
};

}  // namespace rp

using namespace rp;

static void fill_out(const SJob& j, const JobState& st, rp_repair_out& out) {
  fill_repair_out(st, j.plan, out);
}


extern "C" {

size_t rp_server_tables_bytes(uint32_t max_resident) {
  return sup(max_resident * sizeof(Job)) +
         sup(max_resident * sizeof(JobState)) + SALIGN;
}

size_t rp_server_job_bytes(const rp_kernel* k) {
  if (validate_kernel(k) != RP_OK) return 0;
  Plan pl;
  make_plan(k, pl);
  JobInput ji;
  ji.plan = &pl;
  ji.phi0.assign(2 * pl.S, rp_clause{0, 0});
  return sup(engine_job_bytes(ji));
}

rp_status rp_server_create(void* arena, size_t arena_bytes, const rp_repair_opts* opts,
                           uint32_t max_resident, void* stream, void** out) {
  if (!arena || !out || max_resident == 0 || max_resident > (1u << 16)) return RP_ERR_INVALID;
  const rp_repair_opts op = opts ? *opts : rp_repair_opts{0, 1, 1, 0, 0};
  if (op.policy > 1 || op.solver > 1) return RP_ERR_INVALID;
  const size_t tb = rp_server_tables_bytes(max_resident);
  if (arena_bytes < tb) return RP_ERR_WORKSPACE;
  Server* sv = new Server();
  sv->arena = (uint8_t*)arena;
  sv->arena_bytes = arena_bytes;
  sv->opts = op;
  sv->s = (hipStream_t)stream;
  sv->max_resident = max_resident;
  size_t o = 0;
  sv->d_jobs = (Job*)(sv->arena + o); o += sup(max_resident * sizeof(Job));
  sv->d_states = (JobState*)(sv->arena + o); o += sup(max_resident * sizeof(JobState));
  sv->d_active = (uint32_t*)(sv->arena + o); o += SALIGN;
  sv->tables = o;
  sv->alloc.init(o, arena_bytes - o);
  *out = sv;
  return RP_OK;
}

rp_status rp_server_submit(void* srv, const rp_kernel* k, uint64_t job_id) {
  Server* sv = (Server*)srv;
  if (!sv || validate_kernel(k) != RP_OK) return RP_ERR_INVALID;
  std::unique_ptr<SJob> j(new SJob());
  j->id = job_id;
  j->desc.take(k);
  make_plan(&j->desc.k, j->plan);
  j->input.plan = &j->plan;
  j->input.phi0 = option_units(j->plan, sv->opts);
  j->input.policy = sv->opts.policy;
  j->input.max_rounds = sv->opts.max_rounds;
  j->input.solver = sv->opts.solver;
  j->bytes = sup(engine_job_bytes(j->input));
  if (j->bytes > sv->arena_bytes - sv->tables) return RP_ERR_BUDGET;   // can never fit
  j->t_submit = now_s();
  sv->pending.push_back(std::move(j));
  return RP_OK;
}

rp_status rp_server_step(void* srv, uint32_t* n_resident, uint32_t* n_pending) {
  Server* sv = (Server*)srv;
  if (!sv) return RP_ERR_INVALID;
  hipStream_t s = sv->s;
  // 1. admission by footprint, arrival order: the longest prefix of the
  // pending jobs (up to MAX_GROUP) whose group region fits a free range and
  // the free slots
  {
    std::vector<JobInput> group;
    size_t n_take = 0, gbytes = 0, off = 0;
    while (n_take < sv->pending.size() && n_take < MAX_GROUP &&
           sv->resident.size() + n_take < sv->max_resident) {
      group.push_back(sv->pending[n_take]->input);
      const size_t b = sup(engine_group_bytes(group));
      // the smaller group's range goes back first, so the larger one may
      // take its place
      if (n_take) sv->alloc.release(off, gbytes);
      size_t o;
      if (!sv->alloc.alloc(b, o)) {
        group.pop_back();
        // the range just released holds the smaller group again
        if (n_take) (void)sv->alloc.alloc(gbytes, off);
        break;
      }
      off = o;
      gbytes = b;
      n_take++;
    }
    if (n_take) {
      std::vector<PreparedJob> prep;
      const int rc = engine_prepare_group(group, sv->arena + off, gbytes, s, prep, sv->staging);
      if (rc != RP_OK) {
        sv->alloc.release(off, gbytes);
        return (rp_status)rc;
      }
      const uint32_t gid = sv->next_group++;
      sv->groups[gid] = Group{off, gbytes, (uint32_t)n_take};
      for (size_t q = 0; q < n_take; q++) {
        std::unique_ptr<SJob>& j = sv->pending.front();
        j->prep = prep[q];
        j->group = gid;
        sv->resident.push_back(std::move(j));
        sv->pending.pop_front();
      }
    }
  }
  const uint32_t n = (uint32_t)sv->resident.size();
  if (n) {
    // 2. one round over every resident job
    sv->h_jobs.resize(n);
    for (uint32_t q = 0; q < n; q++) sv->h_jobs[q] = sv->resident[q]->prep.job;
    if (hipMemcpyAsync(sv->d_jobs, sv->h_jobs.data(), n * sizeof(Job), hipMemcpyHostToDevice, s) !=
        hipSuccess)
      return RP_ERR_DEVICE;
    const int rc = engine_round(sv->d_jobs, n, sv->d_active, s);
    if (rc != RP_OK) return (rp_status)rc;
    gather_states_kernel<<<(n + 255) / 256, 256, 0, s>>>(sv->d_jobs, n, sv->d_states);
    sv->h_states.resize(n);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(sv->h_states.data(), sv->d_states, n * sizeof(JobState),
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return RP_ERR_DEVICE;
    sv->rounds++;
    // 3. retire
    const double t = now_s();
    std::vector<std::unique_ptr<SJob>> keep;
    keep.reserve(n);
    for (uint32_t q = 0; q < n; q++) {
      std::unique_ptr<SJob>& j = sv->resident[q];
      if (sv->h_states[q].state == ST_RUN) {
        keep.push_back(std::move(j));
        continue;
      }
      Server::Done dn;
      dn.id = j->id;
      fill_out(*j, sv->h_states[q], dn.out);
      dn.latency = t - j->t_submit;
      sv->done.push_back(dn);
      auto g = sv->groups.find(j->group);
      if (g != sv->groups.end() && --g->second.live == 0) {
        sv->alloc.release(g->second.off, g->second.bytes);
        sv->groups.erase(g);
      }
    }
    sv->resident.swap(keep);
  } else if (hipStreamSynchronize(s) != hipSuccess) {
    return RP_ERR_DEVICE;
  }
  if (n_resident) *n_resident = (uint32_t)sv->resident.size();
  if (n_pending) *n_pending = (uint32_t)sv->pending.size();
  return RP_OK;
}

rp_status rp_server_poll(void* srv, uint64_t* ids, rp_repair_out* outs, double* latency_s,
                         uint32_t cap, uint32_t* n_done) {
  Server* sv = (Server*)srv;
  if (!sv || (cap && (!ids || !outs))) return RP_ERR_INVALID;
  uint32_t m = 0;
  while (m < cap && !sv->done.empty()) {
    const Server::Done& dn = sv->done.front();
    ids[m] = dn.id;
    outs[m] = dn.out;
    if (latency_s) latency_s[m] = dn.latency;
    sv->done.pop_front();
    m++;
  }
  if (n_done) *n_done = m;
  return RP_OK;
}

rp_status rp_server_destroy(void* srv) {
  Server* sv = (Server*)srv;
  if (!sv) return RP_ERR_INVALID;
  (void)hipStreamSynchronize(sv->s);
  delete sv;
  return RP_OK;
}

}  // extern "C"

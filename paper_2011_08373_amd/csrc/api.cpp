// The C ABI of librepair (declared in include/librepair.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <thread>
#include <vector>

#include "common.h"
#include "launch.h"
#include "plan.h"

namespace rp {
static thread_local rp_stats t_stats;
constexpr uint32_t TRAJ_CAP = 4096;
extern int g_digit_bits_ref(int v, bool set);
int scatter_variant(int v, bool set);
int scatter_wgs(int v, bool set);
int j0_variant(int v, bool set);
int j0_fields_variant(int v, bool set);
int pass_shapes(int v, bool set);

// The option units of the switches of Section 4.2 (Tab. 3): with grid-level
// barriers disabled every grid slot stays off; with inspection disabled every
// pre-existing barrier stays on.  A pre-existing grid barrier under both
// switches is forced both ways, so such a repair is UNSAT at its first Solve,
// before any Verify call (Alg. 1 solves first).
std::vector<rp_clause> option_units(const Plan& pl, const rp_repair_opts& o) {
  std::vector<rp_clause> u;
  for (uint32_t s = 0; s < pl.S; s++) {
    const uint64_t b = 1ull << s;
    if (!o.grid && (pl.grid_slots & b)) u.push_back(rp_clause{0, b});
    if (!o.inspect && (pl.pre_slots & b)) u.push_back(rp_clause{b, 0});
  }
  std::sort(u.begin(), u.end(), [](const rp_clause& a, const rp_clause& b) {
    return a.pos != b.pos ? a.pos < b.pos : a.neg < b.neg;
  });
  return u;
}

static void worst_units(const Plan& pl, std::vector<rp_clause>& u) {
  u.assign(2 * pl.S, rp_clause{0, 0});
}

// The plans of many kernels (validated first), made on a few host threads
// when there are many: each plan is independent.  plans[j] is valid only
// where ok[j].
static void make_plans(const rp_kernel* const* ks, uint32_t n, std::vector<Plan>& plans,
                       std::vector<uint8_t>& ok) {
  plans.assign(n, Plan{});
  ok.assign(n, 0);
  auto one = [&](uint32_t j) {
    if (validate_kernel(ks[j]) != RP_OK) return;
    make_plan(ks[j], plans[j]);
    ok[j] = 1;
  };
  unsigned nth = std::min<unsigned>(16, std::max(1u, std::thread::hardware_concurrency()));
  if (n < 64 || nth < 2) {
    for (uint32_t j = 0; j < n; j++) one(j);
    return;
  }
  nth = std::min<unsigned>(nth, n / 32);
  std::atomic<uint32_t> next(0);
  auto work = [&]() {
    for (;;) {
      const uint32_t j0 = next.fetch_add(16);
      if (j0 >= n) break;
      for (uint32_t j = j0; j < std::min(n, j0 + 16); j++) one(j);
    }
  };
  std::vector<std::thread> pool;
  for (unsigned t = 1; t < nth; t++) pool.emplace_back(work);
  work();
  for (std::thread& t : pool) t.join();
}

// The result of one repair job from its final device state.
void fill_repair_out(const JobState& s, const Plan& pl, rp_repair_out& out) {
  std::memset(&out, 0, sizeof(out));
  out.rounds = s.rounds;
  out.n_clauses = s.n_phi;
  if (s.state == ST_SAFE) {
    out.status = RP_OK;
    out.assign = s.x;
    out.weight = s.weight;
    out.added = s.x & ~pl.pre_slots;
    out.removed = pl.pre_slots & ~s.x;
  } else if (s.state == ST_UNSAT) {
    out.status = RP_UNSAT;
  } else if (s.state == ST_ROUNDS) {
    out.status = RP_ERR_ROUNDS;
  } else if (s.state == ST_ERROR) {
    out.status = job_error_status(s);
  } else {
    out.status = RP_ERR_DEVICE;
  }
}

}  // namespace rp

using namespace rp;

extern "C" {

const char* rp_status_string(int s) {
  switch (s) {
    case RP_OK: return "ok";
    case RP_UNSAT: return "unsat: the kernel cannot be repaired";
    case RP_ERR_INVALID: return "invalid descriptor or argument";
    case RP_ERR_CAPACITY: return "capacity exceeded";
    case RP_ERR_WORKSPACE: return "workspace too small";
    case RP_ERR_DEVICE: return "device error";
    case RP_ERR_ROUNDS: return "round limit reached";
    case RP_ERR_BUDGET: return "job exceeds the memory budget";
    case RP_ERR_SEARCH: return "search limit: the exact solver's node budget was spent";
    default: return "unknown status";
  }
}

rp_status rp_validate(const rp_kernel* k) { return (rp_status)validate_kernel(k); }

size_t rp_workspace_bytes(const rp_kernel* k, int op) {
  if (validate_kernel(k) != RP_OK || op < RP_OP_CHECK || op > RP_OP_FIRST) return 0;
  Plan pl;
  make_plan(k, pl);
  JobInput ji;
  ji.plan = &pl;
  EngineOpts o;
  o.op = (Op)op;
  if (op == RP_OP_REPAIR) {
    worst_units(pl, ji.phi0);
    o.traj_cap = TRAJ_CAP;
  }
  std::vector<JobInput> v{ji};
  return engine_workspace(v, o);
}

rp_status rp_check(const rp_kernel* k, uint64_t x, rp_pair* pairs, uint64_t cap,
                   uint64_t* n_pairs, uint64_t* divergent, uint64_t* n_records, void* ws,
                   size_t ws_bytes, void* stream) {
  if (validate_kernel(k) != RP_OK || (cap && !pairs)) return RP_ERR_INVALID;
  Plan pl;
  make_plan(k, pl);
  JobInput ji;
  ji.plan = &pl;
  ji.x = x;
  EngineOpts o;
  o.op = OP_CHECK;
  o.pair_cap = cap;
  std::vector<JobInput> v{ji};
  std::vector<JobResult> res;
  rp_stats st;
  int rc = engine_run(v, o, ws, ws_bytes, (hipStream_t)stream, res, &st);
  t_stats = st;
  if (rc != RP_OK) return (rp_status)rc;
  if (res[0].st.state == ST_ERROR) return (rp_status)job_error_status(res[0].st);
  if (n_pairs) *n_pairs = res[0].n_pairs;
  if (res[0].n_pairs > cap) return RP_ERR_CAPACITY;
  if (res[0].n_pairs) std::memcpy(pairs, res[0].pairs.data(), res[0].n_pairs * sizeof(rp_pair));
  if (divergent) *divergent = res[0].st.divergent;
  if (n_records) *n_records = pl.accesses;
  return RP_OK;
}

rp_status rp_clauses(const rp_kernel* k, uint64_t x, rp_clause* out, uint64_t cap,
                     uint64_t* n_out, void* ws, size_t ws_bytes, void* stream) {
  if (validate_kernel(k) != RP_OK || (cap && !out)) return RP_ERR_INVALID;
  Plan pl;
  make_plan(k, pl);
  JobInput ji;
  ji.plan = &pl;
  ji.x = x;
  EngineOpts o;
  o.op = OP_CLAUSES;
  std::vector<JobInput> v{ji};
  std::vector<JobResult> res;
  rp_stats st;
  int rc = engine_run(v, o, ws, ws_bytes, (hipStream_t)stream, res, &st);
  t_stats = st;
  if (rc != RP_OK) return (rp_status)rc;
  if (res[0].st.state == ST_ERROR) return (rp_status)job_error_status(res[0].st);
  const uint64_t n = res[0].phi.size();
  if (n_out) *n_out = n;
  if (n > cap) return RP_ERR_CAPACITY;
  if (n) std::memcpy(out, res[0].phi.data(), n * sizeof(rp_clause));
  return RP_OK;
}

rp_status rp_first_partners(const rp_kernel* k, uint64_t x, uint32_t* first,
                            uint64_t* divergent, void* ws, size_t ws_bytes, void* stream) {
  if (validate_kernel(k) != RP_OK || (k->n_points && !first)) return RP_ERR_INVALID;
  Plan pl;
  make_plan(k, pl);
  JobInput ji;
  ji.plan = &pl;
  ji.x = x;
  EngineOpts o;
  o.op = OP_FIRST;
  std::vector<JobInput> v{ji};
  std::vector<JobResult> res;
  rp_stats st;
  int rc = engine_run(v, o, ws, ws_bytes, (hipStream_t)stream, res, &st);
  t_stats = st;
  if (rc != RP_OK) return (rp_status)rc;
  if (res[0].st.state == ST_ERROR) return (rp_status)job_error_status(res[0].st);
  if (pl.P) std::memcpy(first, res[0].first.data(), 2 * (size_t)pl.P * sizeof(uint32_t));
  if (divergent) *divergent = res[0].st.divergent;
  return RP_OK;
}

static bool solve_args_ok(const rp_clause* c, uint64_t n, const uint32_t* w, uint32_t S) {
  if (S > 64 || (n && !c) || (S && !w) || n > (1u << 20)) return false;
  for (uint32_t s = 0; s < S; s++)
    if (w[s] < 1) return false;
  const uint64_t valid = S >= 64 ? ~0ull : ((1ull << S) - 1);
  for (uint64_t q = 0; q < n; q++)
    if ((c[q].pos | c[q].neg) & ~valid) return false;
  return true;
}

static void solve_plan(uint32_t S, const uint32_t* w, Plan& pl) {
  pl.P = 0;
  pl.S = S;
  pl.B = pl.T = 1;
  pl.weights.assign(w, w + S);
  pl.cnt_pre.assign(1, 0);
  pl.gcnt_pre.assign(1, 0);
}

size_t rp_solve_workspace_bytes(uint64_t n_clauses) {
  Plan pl;
  std::vector<uint32_t> w(64, 1);
  solve_plan(64, w.data(), pl);
  JobInput ji;
  ji.plan = &pl;
  ji.phi0.assign(n_clauses, rp_clause{0, 0});
  EngineOpts o;
  o.op = OP_SOLVE;
  std::vector<JobInput> v{ji};
  return engine_workspace(v, o);
}

rp_status rp_min_barriers(const rp_clause* clauses, uint64_t n_clauses, const uint32_t* weights,
                          uint32_t n_slots, uint64_t* assign, uint64_t* weight, void* ws,
                          size_t ws_bytes, void* stream) {
  if (!solve_args_ok(clauses, n_clauses, weights, n_slots)) return RP_ERR_INVALID;
  Plan pl;
  solve_plan(n_slots, weights, pl);
  JobInput ji;
  ji.plan = &pl;
  ji.phi0.assign(clauses, clauses + n_clauses);
  EngineOpts o;
  o.op = OP_SOLVE;
  std::vector<JobInput> v{ji};
  std::vector<JobResult> res;
  rp_stats st;
  int rc = engine_run(v, o, ws, ws_bytes, (hipStream_t)stream, res, &st);
  t_stats = st;
  if (rc != RP_OK) return (rp_status)rc;
  if (res[0].st.state == ST_ERROR) return (rp_status)job_error_status(res[0].st);
  if (res[0].st.state == ST_UNSAT) return RP_UNSAT;
  if (assign) *assign = res[0].st.x;
  if (weight) *weight = res[0].st.weight;
  return RP_OK;
}

rp_status rp_repair(const rp_kernel* k, const rp_repair_opts* opts, rp_repair_out* out,
                    uint64_t* trajectory, uint32_t traj_cap, void* ws, size_t ws_bytes,
                    void* stream) {
  if (validate_kernel(k) != RP_OK || !out || (traj_cap && !trajectory)) return RP_ERR_INVALID;
  rp_repair_opts op = opts ? *opts : rp_repair_opts{0, 1, 1, 0, 0};
  if (op.policy > 1 || op.solver > 1) return RP_ERR_INVALID;
  Plan pl;
  make_plan(k, pl);
  JobInput ji;
  ji.plan = &pl;
  ji.phi0 = option_units(pl, op);
  ji.policy = op.policy;
  ji.max_rounds = op.max_rounds;
  ji.solver = op.solver;
  EngineOpts o;
  o.op = OP_REPAIR;
  o.traj_cap = TRAJ_CAP;
  std::vector<JobInput> v{ji};
  std::vector<JobResult> res;
  rp_stats st;
  int rc = engine_run(v, o, ws, ws_bytes, (hipStream_t)stream, res, &st);
  t_stats = st;
  if (rc != RP_OK) return (rp_status)rc;
  fill_repair_out(res[0].st, pl, *out);
  if (traj_cap) {
    const size_t nt = std::min<size_t>(traj_cap, res[0].traj.size());
    std::memcpy(trajectory, res[0].traj.data(), nt * sizeof(uint64_t));
  }
  return (rp_status)out->status;
}

size_t rp_batch_workspace_bytes(const rp_kernel* const* ks, uint32_t n) {
  if (!ks) return 0;
  std::vector<Plan> plans;
  std::vector<uint8_t> ok;
  make_plans(ks, n, plans, ok);
  std::vector<JobInput> v;
  v.reserve(n);
  for (uint32_t j = 0; j < n; j++) {
    if (!ok[j]) continue;
    v.emplace_back();
    v.back().plan = &plans[j];
    worst_units(plans[j], v.back().phi0);
  }
  EngineOpts o;
  o.op = OP_REPAIR;
  return engine_workspace(v, o);
}

rp_status rp_repair_batch(const rp_kernel* const* ks, uint32_t n, const rp_repair_opts* opts,
                          rp_repair_out* outs, void* ws, size_t ws_bytes, void* stream) {
  if (!ks || !outs) return RP_ERR_INVALID;
  rp_repair_opts op = opts ? *opts : rp_repair_opts{0, 1, 1, 0, 0};
  if (op.policy > 1 || op.solver > 1) return RP_ERR_INVALID;
  std::vector<Plan> plans;
  std::vector<uint8_t> ok;
  std::vector<uint32_t> idx;
  make_plans(ks, n, plans, ok);
  for (uint32_t j = 0; j < n; j++) {
    // every result reads as a failure until its job has a verdict, so a
    // call that ends early leaves no job looking repaired
    std::memset(&outs[j], 0, sizeof(outs[j]));
    outs[j].status = ok[j] ? RP_ERR_DEVICE : RP_ERR_INVALID;   // invalid: this job only
    if (ok[j]) idx.push_back(j);
  }
  std::vector<JobInput> v(idx.size());
  for (size_t q = 0; q < idx.size(); q++) {
    const Plan& pl = plans[idx[q]];
    v[q].plan = &pl;
    v[q].phi0 = option_units(pl, op);
    v[q].policy = op.policy;
    v[q].max_rounds = op.max_rounds;
    v[q].solver = op.solver;
  }
  if (v.empty()) return RP_OK;
  EngineOpts o;
  o.op = OP_REPAIR;
  std::vector<JobResult> res;
  rp_stats st;
  int rc = engine_run(v, o, ws, ws_bytes, (hipStream_t)stream, res, &st);
  t_stats = st;
  if (rc != RP_OK) return (rp_status)rc;
  for (size_t q = 0; q < v.size(); q++) {
    fill_repair_out(res[q].st, plans[idx[q]], outs[idx[q]]);
  }
  return RP_OK;
}

void rp_last_stats(rp_stats* out) {
  if (out) *out = t_stats;
}

int rp_set_sort_digit_bits(int bits) {
  if (bits != 0 && (bits < 8 || bits > 11)) return -1;
  return g_digit_bits_ref(bits, true);
}

uint32_t rp_sort_key_bits(const rp_kernel* const* ks, uint32_t n) {
  if (n && !ks) return 0;
  uint32_t kb = 0;
  for (uint32_t q = 0; q < n; q++) {
    if (validate_kernel(ks[q]) != RP_OK) return 0;
    Plan pl;
    make_plan(ks[q], pl);
    kb = std::max(kb, pl.key_bits);
  }
  return kb;
}

int rp_set_tuning(int knob, int value) {
  switch (knob) {
    case RP_TUNE_SORT_DIGIT_BITS:
      if (value != 0 && (value < 8 || value > 11)) return -1;
      return g_digit_bits_ref(value, true);
    case RP_TUNE_SCATTER_SHAPE:
      if (value < 0 || value > SCATTER_SHAPE_MAX) return -1;
      return scatter_variant(value, true);
    case RP_TUNE_SCATTER_WGS:
      if (value < 0 || value > 8) return -1;
      return scatter_wgs(value, true);
    case RP_TUNE_TIMING:
      if (value < 0 || value > 2) return -1;
      return timing_level(value, true);
    case RP_TUNE_SOLVER_NODES:
      if (value < 4 || value > 40) return -1;
      return solver_nodes_log2(value, true);
    case RP_TUNE_SCAN_PIPELINE:
      if (value < 0 || value > 1) return -1;
      return j0_variant(value, true);
    case RP_TUNE_DIGIT_ORDER:
      if (value < 0 || value > 1) return -1;
      return digit_order(value, true);
    case RP_TUNE_LOW_DIGIT_BITS:
      if (value != 0 && (value < 6 || value > 9)) return -1;
      return low_digit_bits(value, true);
    case RP_TUNE_SCAN_FIELDS:
      if (value < 0 || value > 1) return -1;
      return j0_fields_variant(value, true);
    case RP_TUNE_PASS_SHAPES:
      if (value < 0 || value > PASS_SHAPES_DEFAULT) return -1;
      for (int p = 0; p < 7; p++) {
        const int v = (value >> (4 * p)) & 15;
        if (v > SCATTER_SHAPE_MAX && v != 15) return -1;
      }
      return pass_shapes(value, true);
    default:
      return -1;
  }
}

}  // extern "C"

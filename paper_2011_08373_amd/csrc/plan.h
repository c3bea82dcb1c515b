// Host-side plan of a kernel model and the multi-job execution engine.
#pragma once
#include <vector>

#include "common.h"

namespace rp {

struct Plan {
  uint32_t P = 0, S = 0, B = 0, T = 0;
  uint32_t tbits = 0, bbits = 0, pbits = 0, nbits = 0, abits = 0, key_shift = 0, key_bits = 0;
  std::vector<DPoint> pts;
  std::vector<uint64_t> wbits;      // bit i: point i writes
  std::vector<uint64_t> bits_any, bits_grid;
  std::vector<uint32_t> weights;
  std::vector<uint64_t> cnt_pre;    // prefix of same-block records per block over points
  std::vector<uint64_t> gcnt_pre;   // prefix of cross-block records over points
  uint64_t div_if_enabled = 0, grid_slots = 0, pre_slots = 0;
  uint32_t pad_array = 0;           // array id of padding records (block conditions)
  uint64_t n_intra = 0, n_inter = 0, accesses = 0;
};

int validate_kernel(const rp_kernel* k);
void make_plan(const rp_kernel* k, Plan& pl);
void compact_words(const rp_kernel* k, Plan& pl);
int pick_digit_bits(uint32_t key_bits);
// One radix pass: it sorts by key bits [lo, lo + bits) above the key shift.
struct DigitPass {
  uint32_t lo, bits;
};
// The radix passes of a key of key_bits bits, in execution order: digits of
// the automatic or set width (RP_TUNE_SORT_DIGIT_BITS), or with the lowest
// digit of RP_TUNE_LOW_DIGIT_BITS bits and the rest split evenly into
// digits of at most 10 bits; highest digit first or lowest first
// (RP_TUNE_DIGIT_ORDER).
std::vector<DigitPass> digit_plan(uint32_t key_bits);
// Width of the lowest digit (RP_TUNE_LOW_DIGIT_BITS, 0 = digits of one
// width); returns the old setting.
int low_digit_bits(int v, bool set);
// hipEvent timing level of engine calls (RP_TUNE_TIMING); returns the old one
int timing_level(int v, bool set);
// Order of the radix passes' digits (RP_TUNE_DIGIT_ORDER: 0 lowest first,
// 1 highest first); returns the old setting.
int digit_order(int v, bool set);
// Node budget of the exact solver's branch and bound (RP_TUNE_SOLVER_NODES,
// as log2); returns the old log2.
int solver_nodes_log2(int v, bool set);
// Library status of a job that ended in ST_ERROR.
int job_error_status(const JobState& st);
struct Plan;
// rp_repair_out of a repair job from its final state.
void fill_repair_out(const JobState& s, const Plan& pl, rp_repair_out& out);
// Unit clauses that the repair options impose before the first Solve.
std::vector<rp_clause> option_units(const Plan& pl, const rp_repair_opts& o);

enum Op { OP_CHECK = 0, OP_CLAUSES = 1, OP_REPAIR = 2, OP_SOLVE = 3, OP_FIRST = 4 };

struct JobInput {
  const Plan* plan;
  uint64_t x = 0;                   // assignment (check / clauses; a repair starts at 0)
  std::vector<rp_clause> phi0;      // initial constraint set (repair: option units)
  uint32_t policy = 0, max_rounds = 0;
  uint32_t solver = 0;              // 0 exact Solve, 1 greedy hitting set (mhs)
};

struct JobResult {
  JobState st;
  std::vector<rp_clause> phi;       // clauses mode: reduced learned clauses
  std::vector<rp_pair> pairs;       // check mode
  std::vector<uint32_t> first;      // first-partner mode: [2][P]
  uint64_t n_pairs = 0;
  std::vector<uint64_t> traj;
};

struct EngineOpts {
  Op op = OP_REPAIR;
  uint64_t pair_cap = 0;            // check: caller's capacity
  uint32_t traj_cap = 0;
  bool want_pairs = true;
  bool use_graph = true;            // capture each round in a hipGraph (non-null stream)
  bool no_alloc = false;            // stage through ordinary host memory, record no
                                    // timing events (no device or page-locked allocation)
};

// Bytes of workspace the engine needs for these jobs.
size_t engine_workspace(const std::vector<JobInput>& jobs, const EngineOpts& o);

// One job prepared in its own device region (serving): a host copy of its
// device job table entry, with absolute device pointers.
struct PreparedJob {
  Job job;
};
size_t engine_job_bytes(const JobInput& job);
// Bytes of one region holding a group of jobs prepared together.
size_t engine_group_bytes(const std::vector<JobInput>& jobs);
// Enqueues upload, record generation, sort, run logs, the first-partner
// tables and the first Solve of a group of jobs into one region, with one
// launch per phase for the whole group; out[j] is job j's device table
// entry.  staging must stay alive until the stream is synced.
int engine_prepare_group(const std::vector<JobInput>& jobs, void* region, size_t bytes,
                         hipStream_t s, std::vector<PreparedJob>& out,
                         std::vector<uint8_t>& staging);
// Enqueues one round (Verify, GenerateClause, Solve, active count) over the
// device table of njobs prepared jobs; *dactive receives the number of jobs
// still running after it.
int engine_round(const Job* djobs, uint32_t njobs, uint32_t* dactive, hipStream_t s);

// Runs the op over all jobs; returns RP_OK or an error status.
int engine_run(const std::vector<JobInput>& jobs, const EngineOpts& o, void* ws, size_t ws_bytes,
               hipStream_t s, std::vector<JobResult>& res, rp_stats* stats);

}  // namespace rp

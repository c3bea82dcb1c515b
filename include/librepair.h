/*
 * librepair -- data-parallel hot path of the counterexample-guided barrier
 * repair loop of Joshi & Muduganti, "GPURepair: Automated Repair of GPU
 * Kernels" (arXiv 2011.08373), for AMD Instinct MI355X (gfx950).
 *
 * The paper repairs a kernel by alternating Solve (a weighted partial MaxSAT
 * query over barrier variables) and Verify (a GPUVerify run) in Alg. 1.  This
 * library computes the concrete counterpart on a finite kernel model: Verify
 * enumerates every thread of every block, so it decides races and barrier
 * divergence exactly for the model; Solve is an exact minimum-weight search.
 *
 * Kernel model (the instrumented program P of Section 2.3):
 *   - `blocks` x `threads` threads; thread (bid, tid);
 *   - arrays: SHARED (one instance per block) or GLOBAL (one instance),
 *     `words` 32-bit words each;
 *   - points 0..n_points-1 in program order after loop unrolling.  An ACCESS
 *     reads or writes `array` at word ((a*tid + b*bid + c) mod words), taken
 *     as the Euclidean residue in [0, words).  A BARRIER is one occurrence of
 *     barrier slot `slot` (barrier variable b_slot, Section 2.2); unrolled
 *     copies of one instrumented barrier share the slot.  NOP does nothing;
 *   - every ACCESS and BARRIER is executed by the threads with
 *     tid % guards[guard].m == guards[guard].r (guard {1,0}: all threads)
 *     of the blocks with bid % block_guards[guard].m ==
 *     block_guards[guard].r (block_guards NULL: every block) -- a branch
 *     on blockIdx;
 *   - slots: level BLOCK (orders the threads of one block) or GRID (orders
 *     every pair of threads, Section 2.2), a pre-existing flag (the
 *     programmer's barrier, which the paper also guards so that it may be
 *     removed) and a weight >= 1 (Section 2.4: gw*gb + lw^ld).
 *
 * Semantics under an assignment x (bit s = barrier variable b_s enabled):
 *   - two access records conflict when they touch the same array instance
 *     and word from two different threads and at least one writes
 *     (Section 1); a same-block pair races unless an enabled barrier of any
 *     level occurs strictly between the two points; a pair from different
 *     blocks (GLOBAL arrays only) races unless an enabled GRID barrier does;
 *   - an enabled BLOCK barrier diverges when some block has 0 < n < threads
 *     of its threads executing it (Section 1, Listing 2); an enabled GRID
 *     barrier diverges when 0 < n < blocks*threads threads of the grid
 *     execute it (a grid barrier must be reached by the whole grid; with
 *     thread-only conditions the two rules agree);
 *   - a race between points i <= j yields the positive clause of the slots
 *     strictly between them (GRID slots only for a cross-block race); a
 *     divergent slot s yields the negative unit {not b_s} (Section 2.4);
 *   - Solve minimises, lexicographically, (total weight, number of enabled
 *     barriers, x as an unsigned integer) over the clauses; the optimum is
 *     unique.
 *
 * Calling convention (every entry point):
 *   - descriptors and output arrays are caller-owned HOST memory, read or
 *     written only during the call;
 *   - `ws` is a caller-owned DEVICE buffer of at least the size returned by
 *     the matching *_workspace_bytes() call, not shared with a concurrent
 *     call; `stream` is a hipStream_t (NULL = default stream).  Work is
 *     ordered on that stream and every call synchronises it before return;
 *   - errors are reported only by the return code.  A validation failure does
 *     no device work.  RP_UNSAT is a result (Alg. 1: the program cannot be
 *     repaired), not a failure.  On RP_ERR_CAPACITY the needed count is
 *     written and nothing else is;
 *   - limits: 1 <= blocks, threads; n_slots <= 64; n_points <= 4096; the
 *     packed access record (array, word, block, point, thread indices) must
 *     fit 64 bits: bits(n_arrays-1) + bits(max words-1) + bits(blocks-1) +
 *     bits(n_points-1) + bits(threads-1) <= 64.
 */
#ifndef LIBREPAIR_H
#define LIBREPAIR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RP_OK = 0,
  RP_UNSAT = 1,             /* Alg. 1: no assignment avoids every trace seen */
  RP_ERR_INVALID = -1,      /* descriptor or argument rejected; no device work */
  RP_ERR_CAPACITY = -2,     /* output (or an internal table) too small */
  RP_ERR_WORKSPACE = -3,    /* ws smaller than the required size */
  RP_ERR_DEVICE = -4,       /* a HIP call or a device-side check failed */
  RP_ERR_ROUNDS = -5,       /* max_rounds Verify calls made without a verdict */
  RP_ERR_BUDGET = -6,       /* server: the job can never fit the memory budget */
  RP_ERR_SEARCH = -7        /* the exact solver's branch and bound spent its node
                               budget (RP_TUNE_SOLVER_NODES) on one component */
} rp_status;

enum { RP_ACCESS = 0, RP_BARRIER = 1, RP_NOP = 2 };
enum { RP_SHARED = 0, RP_GLOBAL = 1 };
enum { RP_BLOCK = 0, RP_GRID = 1 };
enum { RP_OP_CHECK = 0, RP_OP_CLAUSES = 1, RP_OP_REPAIR = 2, RP_OP_FIRST = 4 };

typedef struct { uint32_t words; uint8_t space; } rp_array;              /* 8 B */
typedef struct { uint32_t m, r; } rp_guard;                              /* 8 B */
typedef struct {
  uint8_t kind, is_write;
  uint16_t array, guard, slot;
  int32_t a, b, c;
} rp_point;                                                              /* 20 B */
typedef struct { uint8_t level, preexisting; uint32_t weight; } rp_slot; /* 8 B */
typedef struct {
  uint32_t blocks, threads, n_arrays, n_guards, n_points, n_slots;
  const rp_array* arrays;
  const rp_guard* guards;
  const rp_point* points;
  const rp_slot* slots;
  const rp_guard* block_guards;   /* NULL or [n_guards]: block condition of each guard */
} rp_kernel;

/* clause: satisfied by x iff (x & pos) != 0 or (~x & neg) != 0 */
typedef struct { uint64_t pos, neg; } rp_clause;
/* racing pair of points i <= j; level 0 same block, 1 different blocks */
typedef struct { uint16_t i, j; uint8_t level, pad; } rp_pair;

typedef struct {
  uint8_t policy;     /* 0: learn every race/divergence of a Verify call;
                         1: learn one trace per call (the smallest of
                            divergence < same-block race < cross-block race) */
  uint8_t grid;       /* 0: grid-level barriers disallowed (unit not b_s) */
  uint8_t inspect;    /* 0: pre-existing barriers kept (unit b_s) */
  uint8_t solver;     /* 0: exact Solve every round; 1: the mhs strategy of
                         Section 2.4 -- the greedy minimal hitting set of the
                         positive clauses (most clauses hit per unit weight,
                         ties to the lower slot, then redundant picks dropped
                         in reverse order), the exact optimum in a round where
                         it breaks a clause, and once it is SAFE one exact
                         query; a different optimum is verified in turn and
                         exact Solve continues.  The result equals solver 0's;
                         rounds and trajectory may differ. */
  uint32_t max_rounds;/* Verify calls allowed; 0 = unlimited */
} rp_repair_opts;

typedef struct {
  int32_t status;     /* RP_OK (repaired), RP_UNSAT or an error */
  uint32_t rounds;    /* Verify calls made, the final SAFE one included */
  uint32_t n_clauses; /* size of the reduced constraint set at exit */
  uint32_t pad;
  uint64_t assign;    /* repaired barrier assignment (0 unless RP_OK) */
  uint64_t weight;    /* its total weight */
  uint64_t added;     /* enabled instrumented (not pre-existing) barriers */
  uint64_t removed;   /* pre-existing barriers left disabled */
} rp_repair_out;

/* Timings of the last call made on this thread (hipEvent milliseconds on the
 * call's stream) and the work it did. */
typedef struct {
  double ms_gen, ms_sort, ms_check, ms_clause, ms_solve, ms_total;
  double ms_sort_pass_max;       /* longest single sort pass */
  double ms_sort_kernels;        /* sum of the radix-pass kernel durations */
  double ms_j0;                  /* first partners with no barrier enabled
                                    (once per kernel) */
  uint64_t records;              /* access records generated (both views) */
  uint64_t accesses;             /* (point, block, thread) accesses */
  uint64_t records_scanned;      /* records read by conflict scans */
  uint32_t sort_passes, sort_launches, rounds, conf_launches;
  double ms_upload;              /* descriptor upload before record generation */
  double ms_conf_kernels;        /* duration of the scan kernel over the
                                    sorted logs (first partners or all pairs) */
} rp_stats;

const char* rp_status_string(int status);

/* Checks every rule above; RP_OK or RP_ERR_INVALID. */
rp_status rp_validate(const rp_kernel* k);

/* Device workspace needed by rp_check / rp_clauses / rp_repair (op =
 * RP_OP_*) on this kernel; 0 when the kernel is invalid. */
size_t rp_workspace_bytes(const rp_kernel* k, int op);

/* Verify(P_x) of Alg. 1: every race and every divergent enabled barrier
 * under assignment x.  pairs: up to `cap` racing point pairs in ascending
 * (level, i, j) order; *n_pairs = their number.  *divergent = enabled slots
 * that diverge.  *n_records = (point, block, thread) accesses examined.
 * The kernel is safe under x iff *n_pairs == 0 and *divergent == 0. */
rp_status rp_check(const rp_kernel* k, uint64_t x,
                   rp_pair* pairs, uint64_t cap, uint64_t* n_pairs,
                   uint64_t* divergent, uint64_t* n_records,
                   void* ws, size_t ws_bytes, void* stream);

/* The part of Verify under x that the repair loop uses: for every point i
 * and view (first[i]: same block, first[n_points + i]: different blocks),
 * the smallest point j >= i that races with i, or UINT32_MAX.  Every race
 * (i, j') has j' >= first[i], and its clause contains the clause of
 * (i, first[i]).  Workspace: rp_workspace_bytes(k, RP_OP_FIRST). */
rp_status rp_first_partners(const rp_kernel* k, uint64_t x, uint32_t* first,
                            uint64_t* divergent, void* ws, size_t ws_bytes, void* stream);

/* GenerateClause of Alg. 1 over every trace under x, reduced: sorted by
 * (pos, neg) ascending, duplicates and subsumed clauses removed. */
rp_status rp_clauses(const rp_kernel* k, uint64_t x,
                     rp_clause* out, uint64_t cap, uint64_t* n_out,
                     void* ws, size_t ws_bytes, void* stream);

/* Solve of Alg. 1 (Sections 2.3-2.4): the canonical minimum-weight
 * assignment satisfying every clause.  RP_OK with *assign / *weight, or
 * RP_UNSAT.  n_slots <= 64; weights >= 1; clause literals < n_slots. */
size_t rp_solve_workspace_bytes(uint64_t n_clauses);
rp_status rp_min_barriers(const rp_clause* clauses, uint64_t n_clauses,
                          const uint32_t* weights, uint32_t n_slots,
                          uint64_t* assign, uint64_t* weight,
                          void* ws, size_t ws_bytes, void* stream);

/* The repair loop of Alg. 1: phi starts with the option units; each round
 * solves phi, verifies the solution and learns clauses until SAFE or UNSAT.
 * trajectory (optional, may be NULL) receives the assignment verified in
 * each round, up to traj_cap entries. */
rp_status rp_repair(const rp_kernel* k, const rp_repair_opts* opts,
                    rp_repair_out* out, uint64_t* trajectory, uint32_t traj_cap,
                    void* ws, size_t ws_bytes, void* stream);

/* Batched Alg. 1 over n kernels of any sizes: one launch per phase covers
 * every kernel (records, sort, run logs), each round is one captured hipGraph
 * (when `stream` is not NULL) over every kernel still running, and the host
 * reads one 32-bit count per round.  outs[j] gets kernel j's result exactly
 * as rp_repair would give it, status included: a kernel that fails
 * validation gets RP_ERR_INVALID, one whose constraint set or a table of its
 * own overflows on the device RP_ERR_CAPACITY, one whose exact search spends
 * its node budget RP_ERR_SEARCH -- and the others still run to their
 * verdicts.  Returns RP_OK unless the whole call failed (then every outs[j]
 * not rejected by validation reads RP_ERR_DEVICE).  Workspace:
 * rp_batch_workspace_bytes over the same kernels. */
size_t rp_batch_workspace_bytes(const rp_kernel* const* ks, uint32_t n);
rp_status rp_repair_batch(const rp_kernel* const* ks, uint32_t n, const rp_repair_opts* opts,
                          rp_repair_out* outs, void* ws, size_t ws_bytes, void* stream);

/* Serving (continuous batching).  The arena is caller-owned device memory
 * (e.g. a torch allocation) that the server uses until rp_server_destroy:
 * fixed tables for up to `max_resident` jobs, then first-fit ranges for the
 * resident jobs (records, run logs, clause sets stay there until a job
 * finishes).  rp_server_submit copies the descriptor (RP_ERR_BUDGET when the
 * job's footprint exceeds the arena); rp_server_step admits pending jobs in
 * arrival order while they fit, runs one round of Alg. 1 over every resident
 * job and retires finished ones; rp_server_poll returns finished jobs with
 * their results (as rp_repair gives them) and latency from submission to
 * verdict.  A server is not thread-safe; its calls must not overlap. */
size_t rp_server_tables_bytes(uint32_t max_resident);
size_t rp_server_job_bytes(const rp_kernel* k);
rp_status rp_server_create(void* arena, size_t arena_bytes, const rp_repair_opts* opts,
                           uint32_t max_resident, void* stream, void** server);
rp_status rp_server_submit(void* server, const rp_kernel* k, uint64_t job_id);
rp_status rp_server_step(void* server, uint32_t* n_resident, uint32_t* n_pending);
rp_status rp_server_poll(void* server, uint64_t* job_ids, rp_repair_out* outs,
                         double* latency_s, uint32_t cap, uint32_t* n_done);
rp_status rp_server_destroy(void* server);

/* Instrumentation (Section 2.2) of a structured program into the kernel
 * model above.
 *
 * Program: `functions[0]` is the kernel, the others are device functions it
 * may call.  Each function is a statement list in which IF and LOOP open a
 * region that a matching END closes:
 *   ACCESS   reads (is_write 0) or writes `array` at word
 *            (a*tid + b*bid + c + d*it) mod words, it = iteration of the
 *            innermost enclosing loop at run time (0 outside every loop);
 *   BARRIER  a pre-existing barrier of `level` (RP_BLOCK or RP_GRID);
 *   IF       body runs on the threads with tid % guards[guard].m ==
 *            guards[guard].r of the blocks with bid % block_guards[guard].m
 *            == block_guards[guard].r (block_guards NULL: every block; a
 *            guard of {1, 0} and {1, 0} is a uniform branch) -- nested
 *            branches take the conjunction of both parts;
 *   LOOP     body runs `count` >= 1 times (a uniform trip count);
 *   CALL     runs function `count` (1 <= count < n_functions; no recursion).
 *
 * Instrumented barriers (barrier variables) are placed in the kernel body
 * only: before every ACCESS, before every IF (outside the branch, at its
 * entry point), at the head of every LOOP (first in each iteration) and
 * before every CALL of a function that reaches an ACCESS -- the places
 * Section 2.2 names and its example kernel shows (a callee gets no sites of
 * its own).  Each place gets a BLOCK variable and, when opts->grid is 1, a
 * GRID variable right after it.  Every pre-existing barrier becomes a
 * variable of its own level with `preexisting` = 1; one inside a device
 * function gets one variable per chain of call sites.  Loops are unrolled
 * and calls inlined: the copies of one place are occurrences of one
 * variable.  Weight of a variable: gw*gb + lw^ld (Section 2.4; gb = 1 for
 * GRID, ld = number of enclosing loops, callers' included).
 *
 * Output order: points in execution order; slots numbered by first
 * occurrence; guards (a thread part in guards[], a block part in
 * block_guards[]) numbered by first use, guard 0 = {1, 0} and {1, 0}.  The
 * kernel model is then `{blocks, threads, n_arrays, n_guards, n_points,
 * n_slots, arrays, guards, points, slots, block_guards}` with the program's
 * blocks, threads and arrays.  Output arrays are caller-owned host memory; the needed counts
 * are always written on RP_OK and RP_ERR_CAPACITY (then nothing else is).
 * RP_ERR_INVALID: malformed program (unbalanced regions, an index out of
 * range, recursion, a branch whose conjunction with the enclosing one holds
 * for no thread or needs a modulus >= 2^32, a weight or word offset that
 * overflows) or a model beyond the limits (64 slots, 4096 points).
 * Host-only: no device work, no stream. */
enum { RP_S_ACCESS = 0, RP_S_BARRIER = 1, RP_S_IF = 2, RP_S_LOOP = 3, RP_S_CALL = 4,
       RP_S_END = 5 };
typedef struct {
  uint8_t kind;       /* RP_S_* */
  uint8_t is_write;   /* ACCESS */
  uint8_t level;      /* BARRIER */
  uint8_t pad;
  uint16_t array;     /* ACCESS */
  uint16_t guard;     /* IF */
  uint32_t count;     /* LOOP: trip count; CALL: callee */
  int32_t a, b, c, d; /* ACCESS */
} rp_stmt;                                                               /* 28 B */
typedef struct { uint32_t n_stmts; const rp_stmt* stmts; } rp_function;
typedef struct {
  uint32_t blocks, threads, n_arrays, n_guards, n_functions;
  const rp_array* arrays;
  const rp_guard* guards;
  const rp_function* functions;
  const rp_guard* block_guards;   /* NULL or [n_guards] */
} rp_program;
typedef struct {
  uint8_t grid;       /* 1: GRID variables beside the BLOCK ones (CUDA's
                         grid-level barriers); 0: BLOCK only */
  uint8_t pad[3];
  uint32_t gw, lw;    /* weight parameters; the paper's defaults are 12, 10 */
} rp_instrument_opts;
rp_status rp_instrument(const rp_program* prog, const rp_instrument_opts* opts,
                        rp_guard* guards, rp_guard* block_guards, uint32_t guards_cap,
                        uint32_t* n_guards,
                        rp_point* points, uint32_t points_cap, uint32_t* n_points,
                        rp_slot* slots, uint32_t slots_cap, uint32_t* n_slots);

/* Statistics of the last call made on this thread. */
void rp_last_stats(rp_stats* out);

/* Sort autotuning: digit width of the LSD radix passes (0 = automatic,
 * else 8..11 bits).  Process-wide; returns the previous value.  The
 * automatic width is the narrowest one (8..10 bits) that sorts the key in
 * the fewest passes of at most 10 bits. */
int rp_set_sort_digit_bits(int bits);

/* Bits of the radix sort key of these kernels sorted together (the largest
 * over them; 0 if one is invalid).  The key is the array id and the word,
 * with each array's words rotated so that the ones its accesses can reach
 * start at 0: its width sets the number of radix passes. */
uint32_t rp_sort_key_bits(const rp_kernel* const* ks, uint32_t n);

/* Tuning knobs (process-wide; return the previous value, -1 if rejected):
 *   RP_TUNE_SORT_DIGIT_BITS  0 = automatic, else 8..11;
 *   RP_TUNE_SCATTER_SHAPE    radix-scatter tile: 0 = 512x16, 1 = 256x16,
 *                            2 = 256x32, 3 = 1024x8, 4 = 512x8 (default),
 *                            5 = 1024x4, 6 = 256x8 (threads x records per
 *                            thread), 7 = 512x8, 8 = 1024x8, 9 = 512x16,
 *                            each with streaming (non-temporal) key loads;
 *                            1024x8 tiles (3, 8) take 512x16 for digits
 *                            wider than 9 bits;
 *   RP_TUNE_TIMING           hipEvent timing behind rp_last_stats: 0 = none
 *                            (every ms_* field 0), 1 = the streaming kernels
 *                            (upload, generation, each radix pass and its
 *                            scatter, the first-partner scan, the all-pairs
 *                            scan) and the total (default), 2 = every phase
 *                            (rounds split into check / clause / solve).
 *                            Each event recorded on the stream costs a few
 *                            microseconds of device idle time;
 *   RP_TUNE_SCATTER_WGS      resident workgroups per compute unit of the
 *                            persistent radix scatter: 0 = what the
 *                            occupancy query reports (default), else 1..8;
 *   RP_TUNE_SOLVER_NODES     log2 of the node budget of the exact solver's
 *                            branch and bound on one component of the
 *                            constraint set, per wave of the workgroup that
 *                            searches it (4..40, default 28).  A job whose
 *                            search spends it ends with RP_ERR_SEARCH;
 *   RP_TUNE_SCAN_PIPELINE    first-partner scan: 0 = each wave loads a range
 *                            of records after scanning the one before it,
 *                            1 = the next range's loads are in flight while
 *                            a range is scanned (default);
 *   RP_TUNE_DIGIT_ORDER      the key digit each radix pass sorts by: 0 = the
 *                            lowest first, 1 = the highest first (default).
 *                            Any fixed order keeps every location's records
 *                            together and in generation order; the order of
 *                            the locations in the log differs.  Records in
 *                            generation order share their high digits over
 *                            long stretches, so the highest-first passes
 *                            write long runs and the lowest digit (short
 *                            runs) comes last, when no next-pass digits
 *                            are stored;
 *   RP_TUNE_LOW_DIGIT_BITS   with the automatic digit width: 6..9 = the
 *                            lowest digit has that many bits and the rest
 *                            of the key is split evenly into digits of at
 *                            most 10 bits (default 6; a tile then writes
 *                            runs of about 64 records of the lowest digit
 *                            where consecutive threads touch consecutive
 *                            words), 0 = digits of one width.  Keys too
 *                            short for digits of at least 6 bits above it
 *                            use one width.  The workspace size depends on
 *                            it;
 *   RP_TUNE_SCAN_FIELDS      first-partner scan: 0 = where the thread, block
 *                            and point bits of every job of the call fit in
 *                            32 bits, the point and id fields are taken from
 *                            the low 32 bits of each record with 32-bit
 *                            instructions (default), 1 = always from the
 *                            whole 64-bit record;
 *   RP_TUNE_PASS_SHAPES      radix-scatter tile of each pass: 4 bits per
 *                            pass in execution order (pass i in bits
 *                            4i..4i+3, passes 0..6), each 0..9 as
 *                            RP_TUNE_SCATTER_SHAPE or 15 = the
 *                            RP_TUNE_SCATTER_SHAPE tile; passes from 7 on
 *                            take that tile.  Default 0x0FFFFFFF (every
 *                            pass on it).  A pass whose digit changes
 *                            slowly along its input (the highest, in
 *                            generation order) writes long runs and gains
 *                            from more resident workgroups; one whose digit
 *                            changes fast writes short runs and gains from
 *                            longer tiles, so their best tiles differ. */
enum { RP_TUNE_SORT_DIGIT_BITS = 0, RP_TUNE_SCATTER_SHAPE = 1, RP_TUNE_TIMING = 2,
       RP_TUNE_SCATTER_WGS = 3, RP_TUNE_SOLVER_NODES = 4, RP_TUNE_SCAN_PIPELINE = 5,
       RP_TUNE_DIGIT_ORDER = 6, RP_TUNE_LOW_DIGIT_BITS = 7, RP_TUNE_SCAN_FIELDS = 8,
       RP_TUNE_PASS_SHAPES = 9 };
int rp_set_tuning(int knob, int value);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the repair
 * loop exactly as rp_repair gives it (same arguments, results and statuses),
 * with no workspace argument.  The device workspace is a fixed array of
 * rp_noalloc_scratch_bytes() (64 MiB) that the library holds on every GPU it
 * runs on until the process ends; a kernel whose repair workspace
 * (rp_workspace_bytes(k, RP_OP_REPAIR)) exceeds it is rejected with
 * RP_ERR_WORKSPACE before any device work.  The call makes no device or
 * page-locked allocation (descriptors and results go through ordinary host
 * memory, rounds are launched without a graph, no timing events; host
 * planning uses the heap) and synchronises `stream` before it returns.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (from several host threads or streams) race and must be serialised by
 * the caller.  rp_last_stats is not updated. */
size_t rp_noalloc_scratch_bytes(void);
rp_status rp_repair_noalloc(const rp_kernel* k, const rp_repair_opts* opts,
                            rp_repair_out* out, uint64_t* trajectory, uint32_t traj_cap,
                            void* stream);

#ifdef __cplusplus
}
#endif
#endif

/*
 * CPU oracle for the barrier-repair path (TEST INFRASTRUCTURE ONLY).
 *
 * Plain, slow reference of what the repair path computes (one thread, or
 * independent array instances spread over host threads, or_set_route).
 * Only the test suite, the smoke entry point and the benchmark's CPU-baseline
 * leg may load it; the product library never links or calls it.  It shares
 * no code, header, table or helper with the HIP library: the structs below
 * restate the kernel-model input format field for field because the format
 * is the interface both sides read.
 *
 * Citations name the passages of Joshi & Muduganti, "GPURepair: Automated
 * Repair of GPU Kernels" (arXiv 2011.08373) each function follows.
 */
#ifndef REPAIR_ORACLE_H
#define REPAIR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes (same values as the library's status enum) */
#define OR_OK            0
#define OR_UNSAT         1
#define OR_ERR_INVALID  (-1)
#define OR_ERR_CAPACITY (-2)
#define OR_ERR_ROUNDS   (-5)

typedef struct { uint32_t words; uint8_t space; } or_array;          /* space 0 shared, 1 global */
typedef struct { uint32_t m, r; } or_guard;                          /* tid % m == r */
typedef struct { uint8_t kind, is_write; uint16_t array, guard, slot;
                 int32_t a, b, c; } or_point;                       /* kind 0 access 1 barrier 2 nop */
typedef struct { uint8_t level, preexisting; uint32_t weight; } or_slot;   /* level 0 block 1 grid */
typedef struct {
  uint32_t blocks, threads, n_arrays, n_guards, n_points, n_slots;
  const or_array* arrays; const or_guard* guards;
  const or_point* points; const or_slot* slots;
  const or_guard* block_guards;   /* NULL or [n_guards]: bid % m == r as well */
} or_kernel;
typedef struct { uint64_t pos, neg; } or_clause;
typedef struct { uint16_t i, j; uint8_t level; uint8_t pad; } or_pair;   /* level 0 intra, 1 inter */
/* policy 0 learn every trace, 1 one trace; solver 0 exact Solve every round,
 * 1 greedy minimal hitting set with exact fallback and a final exact query */
typedef struct { uint8_t policy, grid, inspect, solver; uint32_t max_rounds; } or_opts;
typedef struct { int32_t status; uint32_t rounds, n_clauses, pad;
                 uint64_t assign, weight, added, removed; } or_result;

int or_validate(const or_kernel* k);

/* Verify (Alg. 1 Verify; Section 1 race/divergence; Section 2.2 barrier semantics).
 * literal != 0: every pair of access records is compared (tiny kernels only).
 * Pairs are written in (level, i, j) ascending order. */
int or_check(const or_kernel* k, uint64_t x, int literal,
             or_pair* pairs, uint64_t cap, uint64_t* n_pairs,
             uint64_t* divergent, uint64_t* n_records);

/* Route of the location-grouped checker behind or_check (literal = 0),
 * or_clauses, or_full_clauses and or_repair: 0 (default) materialises the
 * records of the whole kernel and groups them at once; 1 takes one array
 * instance at a time -- (array, block) for the same-block relation, (global
 * array, address stripe) for the cross-block one -- on `threads` host
 * threads (0: every core), which bounds memory on the largest workloads.
 * A cross-block part holds about `part_records` records (0: 2^25).  Both
 * routes evaluate the same definition.  Returns the previous route. */
int or_set_route(int route, int threads, uint64_t part_records);

/* Conflict of one pair of points, independent of any assignment. */
int or_pair_conflict(const or_kernel* k, uint32_t i, uint32_t j, int level);

/* GenerateClause over every trace under x, reduced (Alg. 1; Section 2.4). */
int or_clauses(const or_kernel* k, uint64_t x, or_clause* out, uint64_t cap, uint64_t* n);

/* Assignment-independent constraint set: all race clauses and all
 * divergence units of slots that would diverge if enabled. */
int or_full_clauses(const or_kernel* k, or_clause* out, uint64_t cap, uint64_t* n);

/* Reduce a clause list: sort by (pos, neg), drop duplicates and subsumed ones. */
uint64_t or_reduce(or_clause* c, uint64_t n);

/* Solve (Alg. 1 Solve; weighted partial MaxSAT of Section 2.3/2.4) with the
 * canonical tie-break (weight, popcount, mask).  method: 0 auto, 1 exhaustive
 * over all slots (n_slots <= 26), 2 branch and bound. */
int or_min_barriers(const or_clause* c, uint64_t n, const uint32_t* weights,
                    uint32_t n_slots, int method, uint64_t* assign, uint64_t* weight);

/* Greedy minimal hitting set of the positive clauses (Section 2.4, mhs
 * strategy); OR_UNSAT on an empty clause. */
int or_greedy_mhs(const or_clause* c, uint64_t n, const uint32_t* weights,
                  uint32_t n_slots, uint64_t* assign);

/* The repair loop of Alg. 1.  trajectory (optional) receives x_r per round. */
int or_repair(const or_kernel* k, const or_opts* o, or_result* out,
              uint64_t* trajectory, uint32_t traj_cap);

/* Safe(x) by brute force over every record pair (tiny kernels). */
int or_safe_literal(const or_kernel* k, uint64_t x);

#ifdef __cplusplus
}
#endif
#endif

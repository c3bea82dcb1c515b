// Internal device-side data layout of librepair (not part of the public ABI).
//
// Access records are packed 64-bit integers.  With field widths tb = bits of
// (threads-1), bb = bits of (blocks-1), pb = bits of (points-1), nb = bits of
// (max words-1), ab = bits of (arrays-1):
//
//   same-block view  (one record per (point, block, thread) access, up to
//                     the reductions below):
//       [ array | word | block | point | thread ]
//   cross-block view (GLOBAL arrays only):
//       [ array | word | point | block | 0...0  ]
//
// The sort key is the top field pair (array, word) at key_shift =
// tb + bb + pb.  Records are generated in increasing order of their low
// fields (block-major for the same-block view, point-major for the
// cross-block view), so a stable radix sort on the key bits, one digit per
// pass, leaves the records of each memory location together and in that
// order (with the lowest digit first the whole log is sorted as plain 64-bit
// integers; another digit order only changes the order of the locations,
// which no scan depends on).  Inside one memory location the
// records are then ordered by point, which is program order: the interval
// between two enabled barriers is a contiguous run for every assignment, so
// the log is sorted once per kernel and rescanned per Verify call.
//
// Records that cannot change a run-log entry are not generated.  What a
// Verify call needs from the records of one point at one location is its
// first id and whether there are two or more ids (threads in the same-block
// view, blocks in the cross-block view).  Hence:
//   - same-block view, word independent of the thread: the first two
//     executing threads of each block (all threads share one word);
//   - cross-block view, word independent of the thread: one record per
//     block (the thread is not part of a cross-block record);
//   - cross-block view, word independent of the block: blocks 0 and 1 only
//     (first id 0; a second id exactly when there are two blocks or more);
//   - one block: no cross-block view (a race needs two blocks).
// Records are still emitted in increasing order of their low fields.
//
// Block conditions (a guard that also tests bid % bm == br): the same-block
// view keeps one fixed record count per block, and a block that does not
// execute a point holds padding records in its place: array id pad_array
// (one past the kernel's arrays, so the array field may take one more bit),
// word 0, that block, that point, thread 0.  They form locations of their
// own with a single id, so they never conflict.  The cross-block view holds
// the executing blocks only.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/librepair.h"

namespace rp {

constexpr uint32_t NONE32 = 0xFFFFFFFFu;
constexpr int MAX_POINTS = 4096;
constexpr int MAX_SORT_PASSES = 8;

// flags of DPoint::flags.  PF_TCONST: the word does not depend on the thread
// (a = 0 mod words); PF_BCONST: it does not depend on the block (b = 0 mod
// words).
constexpr uint8_t PF_WRITE = 1, PF_GLOBAL = 2, PF_POW2 = 4, PF_TCONST = 8, PF_BCONST = 16;

struct DPoint {          // 40 B, one per program point
  int32_t a, b, c;
  uint32_t words;        // array size (words)
  uint32_t m, r;         // guard: tid % m == r
  uint32_t cnt;          // threads of one block executing the point
  uint16_t array;
  uint8_t kind;          // RP_ACCESS / RP_BARRIER / RP_NOP
  uint8_t flags;         // PF_*
  uint32_t bm, br;       // block condition: bid % bm == br
};

struct JobState {        // device-resident per-job state; the host reads it
  uint64_t x;            // current assignment
  uint64_t weight;       // weight of x
  uint64_t divergent;    // enabled divergent slots at the last Verify
  uint32_t n_phi;        // clauses in phi (reduced)
  uint32_t state;        // 0 running, 1 safe, 2 unsat, 3 error
  uint32_t rounds;       // Verify calls made
  uint32_t races;        // (point, level) rows with a race at the last Verify
  uint32_t err;          // device-side error code (0 = none)
  uint32_t max_rounds;   // 0 = unlimited
  uint64_t traj_pad;
  uint32_t phase;        // PH_*: which Solve the next call makes
  uint32_t pad3;
};
constexpr uint32_t ST_RUN = 0, ST_SAFE = 1, ST_UNSAT = 2, ST_ERROR = 3, ST_ROUNDS = 4;
// Solve phases.  PH_EXACT: the exact optimum.  PH_GREEDY (mhs strategy,
// until the first SAFE): the greedy hitting set of the positive clauses, the
// exact optimum when it leaves a clause unsatisfied.  PH_FINAL: the verified
// greedy answer is SAFE; one exact query either confirms it or replaces it,
// and exact Solve continues.
constexpr uint32_t PH_EXACT = 0, PH_GREEDY = 1, PH_FINAL = 2;
// device-side error codes of a job (JobState::err) or of a whole call (the
// error word): phi or a scratch table full, an out-of-range sort output, the
// exact solver's node budget spent
constexpr uint32_t ERR_PHI_CAP = 1, ERR_SORT = 2, ERR_SCRATCH = 3, ERR_RANGE = 4, ERR_NODES = 5;

struct Job {
  uint32_t P, S, B, T;
  uint32_t tbits, bbits, pbits, key_shift;
  uint32_t nbits, policy;     // word-field width; learning policy
  const DPoint* pts;          // [P]
  const uint64_t* wbits;      // [(P+63)/64] bit i: point i writes
  const uint64_t* bits_any;   // [P] slot bit of a barrier occurrence, else 0
  const uint64_t* bits_grid;  // [P] slot bit of a GRID barrier occurrence, else 0
  const uint32_t* weights;    // [S]
  const uint64_t* cnt_pre;    // [P+1] prefix of same-block records per block
  const uint64_t* gcnt_pre;   // [P+1] prefix of cross-block records
  uint64_t rblk;              // same-block records per block (= cnt_pre[P])
  uint64_t div_if_enabled;    // slots whose guard splits a block
  const uint64_t* log[2];     // sorted logs: same-block, cross-block
  uint64_t nlog[2];
  uint32_t* ivl;              // [2][P] interval id: any level, grid level
  uint32_t* minj;             // [2][P] first racing partner per point under x
  uint32_t* j0;               // [2][P] first racing partner with no barrier enabled
  uint64_t* bitmap;           // [2][P][wpr] racing pairs (check mode) or null
  uint32_t wpr;               // 64-bit words per bitmap row
  uint32_t pad_array;         // array id of padding records (0: none)
  rp_clause* phi;             // [phi_cap]
  rp_clause* scratch;         // [scratch_cap] (power of two)
  uint32_t phi_cap, scratch_cap;
  JobState* st;
  uint64_t* traj;             // [traj_cap] assignment verified per round
  uint32_t traj_cap, pad2;
  uint64_t node_limit;        // nodes the exact solver's branch and bound may visit
};

// sort segment: one log of one job in the record buffer
struct SortSeg {
  uint64_t beg, end;     // record range
  uint32_t shift;        // key_shift of the job
  uint32_t chunk_beg, chunk_end;  // its chunks
  uint32_t job, view;    // the job and log (0 same-block, 1 cross-block)
  uint32_t cblk_beg;     // its first column block (COL_BLOCK_CHUNKS chunks each)
};

// Chunks per column block: the column scans of a pass read and write the
// per-chunk digit tables a block of chunks at a time, every row whole.
constexpr uint32_t COL_BLOCK_CHUNKS = 32;

// sort chunk: a record range inside one segment, one workgroup per pass
struct SortChunk {
  uint64_t beg, end;
  uint32_t seg, pad;
};

// generation work item: records [o0, o1) of one log (segment-local indices)
struct GenItem {
  uint64_t o0, o1;
  uint32_t job, view;    // view 0 same-block log, 1 cross-block log
  uint32_t seg, i0;      // i0: the point holding record o0
};

// one log of one job: its sorted records
struct ConfSeg {
  const uint64_t* log;   // sorted access records
  uint64_t n;            // records
  uint32_t job, level;   // level 0 same-block view, 1 cross-block view
  uint32_t ctile_beg;    // first record tile of the scan (set on the device)
  uint32_t pad;
};

// Scan entry (64 bits) of one record of a sorted log, in location order and,
// inside a location, in program order:
//   bits  0..31  id: the thread (same-block view) or the block (cross-block view)
//   bits 32..43  point
//   bit  44      the point writes
//   bit  45      first record of a streak: first of its location, or its id
//                differs from the previous record's
//   bit  46      first record of its location
//   bit  47      never set in an entry: marks the sentinel read past a log
constexpr int RUN_PT = 32, RUN_W = 44, RUN_X = 45, RUN_LOC = 46, RUN_END = 47;
constexpr uint64_t RUN_SENTINEL = (1ull << RUN_X) | (1ull << RUN_LOC) | (1ull << RUN_END);

__device__ __forceinline__ uint32_t word_of(const DPoint& p, uint32_t t, uint32_t k) {
  int64_t v = (int64_t)p.a * (int64_t)t + (int64_t)p.b * (int64_t)k + (int64_t)p.c;
  if (p.flags & PF_POW2) return (uint32_t)((uint64_t)v & (uint64_t)(p.words - 1));
  int64_t n = (int64_t)p.words;
  int64_t r = v % n;
  return (uint32_t)(r < 0 ? r + n : r);
}

// radix digit of a record for a pass starting at bit `shift` (0 past bit 63)
__device__ __forceinline__ uint32_t digit_at(uint64_t rec, int shift, uint32_t mask) {
  return shift < 64 ? (uint32_t)(rec >> shift) & mask : 0u;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  uint32_t lane = __lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Global-memory view of a pointer read from a device table.  The compiler
// must use flat instructions for a pointer of unknown address space, and a
// flat load also counts against the LDS wait counter: every wait for it then
// waits for all LDS operations too, and a wait for an LDS result waits for
// every load in flight.  Loads through this view are global loads.
template <typename T>
using gptr = const __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> as_global(const T* p) {
  return (gptr<T>)p;
}

}  // namespace rp

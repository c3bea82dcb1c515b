// Launchers of the device kernels (one per .hip file), called by the host
// library.  All return the launch status; none synchronises.
#pragma once
#include "common.h"

namespace rp {

uint32_t sort_tile_size();
uint32_t conf_tile_size();

// count_lo: generation stores per-chunk counts of key bits [count_lo,
// count_lo + rb) (the first pass's digit) in item_hist; -1 for none
hipError_t launch_gen(int rb, const GenItem* items, uint32_t n_items, const Job* jobs,
                      const SortSeg* segs, uint64_t* recs, uint32_t* item_hist, int count_lo,
                      hipStream_t s);
// generation items and sort chunks: chunk c of segment s covers its records
// [(c - chunk_beg) * chunk_len, ...) up to the segment's end
hipError_t launch_items(const Job* jobs, const SortSeg* segs, uint32_t nseg, uint32_t nchunks,
                        uint64_t chunk_len, GenItem* items, SortChunk* chunks, hipStream_t s);
// dig: each record's digit of this pass (1 byte for 8-bit digits, else 2),
// as the previous pass's scatter wrote it; unused when counts_ready (pass 0
// takes its counts from record generation)
// n_cblk column blocks over all segments (each segment's from its cblk_beg),
// at most max_cblk in one segment; part: [n_cblk][2^rb] scratch
hipError_t launch_sort_scan(int rb, const void* dig, const SortSeg* segs, uint32_t nseg,
                            const SortChunk* chunks, uint32_t nchunks, uint32_t n_cblk,
                            uint32_t max_cblk, uint32_t* cnt, uint64_t* tot, uint64_t* part,
                            uint64_t* off, uint32_t* ticket, bool counts_ready, hipStream_t s);
// The pass sorts by key bits [lo, lo + rb) above each segment's key shift;
// the next pass's digit, key bits [nlo, nlo + nbits), is stored per output
// record in dnext (1 byte for up to 8 bits, else 2; NULL after the last
// pass); ticket: one device word, set to zero by launch_sort_scan of the
// same pass; pass: the pass's index in execution order (its tile shape)
hipError_t launch_sort_scatter(int rb, int pass, const uint64_t* in, uint64_t* out,
                               const SortSeg* segs, const SortChunk* chunks, uint32_t nchunks,
                               int lo, int nlo, int nbits, const uint64_t* off, uint32_t* ticket,
                               uint32_t* err, void* dnext, hipStream_t s);
// Radix-scatter tile shapes 0..SCATTER_SHAPE_MAX; the per-pass shapes'
// default (every pass on the common shape)
constexpr int SCATTER_SHAPE_MAX = 9;
constexpr int PASS_SHAPES_DEFAULT = 0x0FFFFFFF;
constexpr int IVL_RESOLVE = 0, IVL_CHECK = 1, IVL_ZERO = 2;
hipError_t launch_ivl(const Job* jobs, uint32_t njobs, int mode, hipStream_t s);
hipError_t launch_save_j0(const Job* jobs, uint32_t njobs, hipStream_t s);
// Lays out the round's tiles over the logs of running jobs: ctile_beg of
// each segment, the total in *tiles.
hipError_t launch_conf_tiles(const Job* jobs, ConfSeg* segs, int nseg, uint32_t* tiles,
                             hipStream_t s);
// Every racing pair under x over the tiles laid out by launch_conf_tiles.
hipError_t launch_conf(const Job* jobs, const ConfSeg* segs, int nseg, uint32_t max_points,
                       const uint32_t* tiles, hipStream_t s);
// First partners with no barrier enabled, into minj (cleared beforehand).
// lo32: the point and id fields of every record lie in its low 32 bits
// (thread, block and point bits together at most 32, in every job)
hipError_t launch_j0(const Job* jobs, const ConfSeg* segs, int nseg, uint32_t max_points,
                     bool lo32, const uint32_t* tiles, hipStream_t s);
hipError_t launch_pairs(const Job* job, rp_pair* out, uint64_t* total, hipStream_t s);
hipError_t launch_clause(const Job* jobs, uint32_t njobs, int learn, hipStream_t s);
hipError_t launch_solve(const Job* jobs, uint32_t njobs, hipStream_t s);
hipError_t launch_count_active(const Job* jobs, uint32_t njobs, uint32_t* out, hipStream_t s);

}  // namespace rp

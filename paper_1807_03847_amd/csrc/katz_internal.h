// Internal declarations shared by the kernels and the host runtime.
//
// Layout of a ranking run on the device
//   * Rows are binned by length (degree-binned scheduling).  Each bin holds
//     RowDesc records {offset, row, length} in ascending row order.  A bin has a
//     fixed number of lanes per row, so the summation order of every row, and
//     therefore its floating-point result, depends only on the row's length.
//   * Rows longer than kBlockRowMax are cut into segments of kSeg arcs; one
//     workgroup sums a segment, and a second launch (one wave per row) adds a
//     row's partials in segment order.  The kernel boundary orders the two,
//     so no device-scope fence is needed between workgroups (on a multi-XCD
//     part such a fence writes back or invalidates a whole L2).
//   * The first walk step (x_0 = 1) sums no vector: row v's sum is its length.
//   * The walk vector is double-buffered; c (FP64) is updated in place; the
//     FP32 form adds the per-node margin accumulator e (FP32, rounded up).
//   * The active set M is a compacted list of node ids, double-buffered.  The
//     top-k threshold is found by an MSB-first radix select on the IEEE bit
//     pattern of the lower bound (non-negative, so the bit order is the value
//     order), 12 bits per digit.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "katz.h"

namespace katz {

constexpr int kWG = 256;                 // threads per workgroup (4 waves of 64)
constexpr int kXcds = 8;
constexpr int kWalkGroups = 4;           // 256-thread groups per workgroup of walk_step_grouped                 // XCDs of an MI355X; workgroups go to them round-robin by id
constexpr int kWave = 64;
constexpr int kPerLane = 16;             // max row elements summed serially per lane
constexpr int kSeg = kWG * kPerLane;     // arcs per huge-row segment (4096)
constexpr int kWaveRowMax = kWave * kPerLane;   // 1024
constexpr int kShortRowMax = 128;               // 16 lanes x 8 elements
constexpr int kBlockRowMax = kSeg;              // 4096
constexpr int kDigitBits = 12;
constexpr int kDigits = 1 << kDigitBits;        // histogram bins per radix digit
constexpr int kSelectLevels = 6;                // digits of a 63-bit key: 12*5 + 3
constexpr int kMaxK = 4096;                     // LDS sort capacity of the check
constexpr int kFinishThreads = 1024;
constexpr int kSmallCand = 16384;               // finish directly below this many

enum BinId : int {
  BIN_HUGE = 0,   // len > 4096: segmented, multi-workgroup
  BIN_B256,       // 1025..4096: one workgroup per row
  BIN_W64,        // 129..1024: one wave per row
  BIN_W16,        // 33..128
  BIN_G32,        // 17..32
  BIN_G16,        // 9..16
  BIN_G8,         // 5..8
  BIN_G4,         // 1..4
  BIN_EMPTY,      // 0
  NUM_BINS
};

// Lanes that sum one row of each bin (lane l adds elements l, l+G, ... in
// order, then the lanes combine by butterfly).  Short rows take few lanes, at
// most eight elements each (one batch of loads), so a wave holds many rows;
// each lane then has eight loads in flight.  The schedule, and so every row
// sum's rounding, depends only on the row's bin.
constexpr int kBinLanes[NUM_BINS] = {kWG, kWG, 64, 16, 4, 2, 1, 1, 1};   // empty rows: one thread each
// Rows per workgroup-sized group of a short-row bin.
constexpr int bin_rows_per_group(int bin) { return kWG / kBinLanes[bin]; }

// Longest row of each length class below BIN_B256 (a row goes to the first
// class whose bound it does not exceed; BIN_B256 ends at kBlockRowMax, longer
// rows are segmented).  The bounds decide how many lanes sum a row, so they
// fix the order of its additions; katz_tuning.bin_bounds sets them.
struct BinBounds {
  int g4 = 4, g8 = 8, g16 = 16, g32 = 32, w16 = kShortRowMax, w64 = kWaveRowMax;
};

struct RowDesc {
  int64_t off;
  int32_t row;
  int32_t len;
};

struct SegDesc {
  int64_t off;
  int32_t len;
  int32_t part;   // index of this segment's partial sum
  int32_t hrow;   // index of the owning row in the huge-row table
  int32_t pad;
};

// Renumbering table, indexed by caller id: the node's internal id and its row
// length (the length gives x_1 of the node, as the first walk step sums ones).
struct IdLen {
  int32_t id;
  int32_t len;
};

struct HugeRow {
  int32_t row;
  int32_t len;
  int32_t nseg;
  int32_t part0;  // partials part0 .. part0 + nseg - 1, in segment order
};

// Device-resident scalars of one run.
struct RunScalars {
  int err;            // CSR validation failure
  int done;           // the run has stopped (every later kernel returns at once)
  int status;         // KATZ_OK or a warning
  int iterations;     // r of the last completed iteration
  int m;              // |M|: length of the current active list
  int top_count;      // top-k nodes appended by the apply kernel
  int kept_count;     // non-top nodes kept active
  int progress;       // FP32 form: some active interval can still shrink
  int cand_count[2];  // candidates compacted at select levels 0 and 1
  int need;           // rank still to find inside the current bucket
  int level;          // select digits resolved so far
  int cut_ext;        // ties with key == theta_key are top iff ext id <= cut_ext
  int fail;           // adjacent-pair test failed
  int dmax;           // prep: maximum row length
  int cur;            // active-list buffer written by the last completed check
  unsigned long long prefix;     // resolved high bits of the k-th key
  unsigned long long theta_key;  // bit pattern of l(M[k])
  double theta;                  // l(M[k])
  long long bin_count[NUM_BINS];
  long long bin_base[NUM_BINS];
  long long seg_total;
  // Walk step 2 of a renumbered run found a caller column id out of range.
  // Kept apart from err while that kernel runs: every wave of a walk kernel
  // reads err once to decide whether to skip its work, and the waves of one
  // workgroup must decide alike (they meet at barriers).  fold_col_err copies
  // it into err after the launch.
  int col_err;
  // An FP32 state's re-walk wrote an entry above its limit (its stored scales
  // no longer fit the graph): the update re-runs the state from level 1.
  int rescale;
};

// Bound evaluation parameters of one iteration.
struct BoundArgs {
  const double* c;
  const void* x;          // double* (FP64) or float* (FP32)
  const float* e;         // FP32 form margin accumulator
  const double* sigma;    // FP32 form: per-iteration scale sigma_r (device)
  const double* sigma_sum;
  int r;
  int fp32;
  int undirected;
  int pad;
  double alpha;
  double beta;            // FP64: fl(alpha * gamma); FP32: upward-rounded beta
  double eps;
  // FP32 widening factors (see bound_eval):
  double f_lo_c, f_hi_c, f_lo_s, f_hi_s, f_e, tau_coef, kappa;
};

struct IterArgs {
  const RowDesc* desc;
  const int32_t* col;
  const SegDesc* segs;
  const HugeRow* huge;
  long long first_block[NUM_BINS + 1];  // fused-launch block ranges per bin
  long long bin_base[NUM_BINS];
  long long bin_count[NUM_BINS];
  const void* x_in;
  void* x_out;
  double* c;
  float* e;
  void* partial;
  void* blkmax;                  // per-workgroup maximum of the new walk entries
  long long blk_base;            // first slot of this launch's workgroup maxima in blkmax
  unsigned* xmax32;              // [max_iter + 1] float bits of max x~_r
  unsigned long long* xmax64;    // [max_iter + 1] double bits of max s_r
  double* sigma;                 // [max_iter + 1]
  double* sigma_sum;             // [max_iter + 1]
  RunScalars* sc;
  int n;
  int r;
  int count_first;               // walk_first: number of descriptors to process
  int write_empty;
  int clog2_dmax;
  int rewalk;                    // dynamic re-walk: write x only (no c, no maxima)
  int hub_n;                     // walk entries 0 .. hub_n - 1 are read from an LDS copy
  double alpha;
  double etap;                   // eta'_r
  // Walk step 2 fused with the internal renumbering (walk_step<F32, true>):
  // each row's caller column ids (col_src + coff[row]) are renamed through
  // pmap and written to col (at desc.off), and a gathered neighbour's x_1 is
  // computed from its length in pmap instead of being read from x_in.
  const int32_t* col_src;
  const long long* coff;         // internal id -> offset of its row in col_src
  const IdLen* pmap;             // caller id -> {internal id, row length}
  int32_t* ncol;                 // renamed column ids (written)
  // Two-pass walk step (hot_n > 0): pass 1 sums each row's entries with column
  // id below hot_n into hot_part (long-row segments: into their partial);
  // pass 2 sums the other entries, adds the pass-1 sum, and runs the epilogue.
  // pass 0: one pass over every entry.
  int pass;
  int hot_n;
  void* hot_part;                // [n] per-row pass-1 sums (FP32 or FP64 as x)
};

struct SelArgs {
  BoundArgs b;
  const int32_t* act_in;
  int32_t* act_out;
  unsigned long long* keys;
  unsigned long long* cand_key[2];
  int32_t* cand_v[2];
  unsigned* hist;                // [2][kDigits]
  const int32_t* ext_of;         // internal -> external id (nullptr: identity)
  const int32_t* int_of;         // external -> internal id (nullptr: identity)
  int32_t* top_sorted;           // [k] internal ids in ranking order
  double* top_lo;
  double* top_up;
  const unsigned* xmax32;
  const unsigned long long* xmax64;
  RunScalars* sc;
  int identity_in;               // first selection of a run: the active list is 0..n-1
  int k;
  int n;
  int max_iter;
  int act_out_idx;               // which active-list buffer act_out is (recorded on completion)
  int pad;
};

// One graph's view for the one-workgroup selection (select_wg): every array
// points at the graph's own region; node ids are global (base .. base + n).
struct GraphSel {
  BoundArgs b;                   // with a device iteration counter, r and x are refreshed
  const void* xbuf[2];           // walk vector buffers by parity of r (device-counter mode)
  const double* etap;            // FP32 form: eta'_r table (device-counter mode)
  const int32_t* act[2];         // active-list buffers of this graph
  unsigned long long* keys;
  unsigned long long* cand_key;
  int32_t* cand_v;
  int32_t* top_sorted;
  double* top_lo;
  double* top_up;
  RunScalars* sc;
  const unsigned* xmax32;        // indexed by r
  const unsigned long long* xmax64;
  const int32_t* ext_of;         // internal -> caller id (nullptr: identity); ties go by caller id
  const int32_t* int_of;         // caller id -> internal id
  int base;
  int n;
  int k;
  int max_iter;
  int identity_in;               // the active list is base .. base + n - 1
  int cur;                       // host-driven mode: buffer holding M (act[cur])
};

// The batched walk step (many graphs, global row ids).
struct BatchWalk {
  const RowDesc* desc;
  const SegDesc* segs;
  const HugeRow* huge;
  long long first_block[NUM_BINS + 1];
  long long bin_base[NUM_BINS];
  long long bin_count[NUM_BINS];
  const int* gid_of;
  const int32_t* const* gcol;
  const long long* gbase;
  const double* galpha;
  const RunScalars* gsc;        // per graph: done / err
  const double* gsigma;         // [count][stride] FP32 scale sigma_r
  const int* gexp;              // [count][stride] exponent e_r
  unsigned* gxmax32;            // [count][stride]
  unsigned long long* gxmax64;  // [count][stride]
  void* xbuf[2];
  double* c;
  float* e;
  void* partial;
  const double* etap;           // eta'_r per graph: [count][stride]
  const int* r_dev;
  const int* item_g;            // per work item: the graph of all its rows, or -1 (rows of several graphs)
  const int* items;             // work items of this iteration (live graphs only), n_items[x] in list x
  const int* n_items;           // [kXcds]
  int* blk_g;                   // per workgroup: graph of all its rows, or -1
  double* blk_m;                // per workgroup: maximum new walk entry of that graph
  long long blk_base;           // first slot of this launch in blk_g / blk_m
  int count;                    // graphs in the batch
  int direct_max;               // 1: workgroups update per-graph maxima with atomics
  int tile;                     // row groups per work item in the short-row bins
  int xcd_groups;               // 1, or kXcds: work-item lists per XCD (items + x * item_cap)
  long long item_cap;           // capacity of one work-item list
  const int* xcd_of;            // per graph: the XCD whose workgroups take its items
  int stride;
  int fp32;
};

// ---- launchers (katz_kernels.hip) ----------------------------------------
hipError_t launch_prep_count(const void* row_ptr, int row_ptr_64, int64_t n, int64_t nnz,
                             long long* blk, int nblocks, RunScalars* sc, const BinBounds& bb, hipStream_t s);
hipError_t launch_prep_scan(long long* blk, int nblocks, long long* sums, long long* totals, RunScalars* sc,
                            hipStream_t s);
hipError_t launch_prep_scatter(const void* row_ptr, int row_ptr_64, int64_t n,
                               const long long* blk, int nblocks, RowDesc* desc,
                               SegDesc* segs, HugeRow* huge, RunScalars* sc, const BinBounds& bb,
                               hipStream_t s);
// segs / nseg / huge: the bins' segments of rows longer than kBlockRowMax
// (their symmetry is checked segment by segment).
hipError_t launch_validate_strict(const RowDesc* desc, long long n, const SegDesc* segs, long long nseg,
                                  const HugeRow* huge, const int32_t* col, int undirected, long long* row_off,
                                  int* row_len, RunScalars* sc, hipStream_t s);
hipError_t launch_walk_first(const IterArgs& a, int fp32, long long n, long long nnz, int validate,
                             hipStream_t s);
// Workgroups of `block` threads and `lds` dynamic LDS bytes of a kernel that
// the device holds at once.
long long resident_blocks(const void* kernel, size_t lds, int block);
long long batch_walk_resident(int fp32);
// renumber: walk step 2 fused with the renaming of the column ids (the
// IterArgs renumbering fields must be set and hub_n must be 0).  groups: 1, or
// kWalkGroups for walk_step_grouped (not with renumber).
hipError_t launch_walk_step(const IterArgs& a, int fp32, long long total_blocks, long long max_grid,
                            long long* grid_used, hipStream_t s, bool renumber = false, int groups = 1);
// Reduces the per-workgroup maxima of walk iteration r into xmax32[r] / xmax64[r].
hipError_t launch_reduce_blkmax(const void* blkmax, long long nb, int fp32, unsigned* xmax32,
                                unsigned long long* xmax64, int r, const RunScalars* sc, hipStream_t s);
hipError_t launch_check_col_range(const int32_t* col, long long nnz, long long n, RunScalars* sc, hipStream_t s);
// sort_key / sort_ext (k elements each): when set, the top-k is sorted and
// tested device-wide (launch_large_check) instead of in one workgroup's LDS.
hipError_t launch_select_iteration(const SelArgs& a, int grid, hipStream_t s,
                                   unsigned long long* sort_key = nullptr, int32_t* sort_ext = nullptr);

// ---- stopping criteria beyond the LDS top-k test (katz_criteria.hip) ------------
hipError_t launch_large_check(const SelArgs& a, unsigned long long* key, int32_t* ext, hipStream_t s);
hipError_t launch_score_check(const SelArgs& a, hipStream_t s);
// Every node (identity list) sorted into top_sorted / top_lo / top_up.
hipError_t launch_score_output(const SelArgs& a, unsigned long long* key, int32_t* ext, hipStream_t s);
hipError_t launch_pair_check(const SelArgs& a, int ext_a, int ext_b, hipStream_t s);
hipError_t launch_separated_count(const double* lo_desc, const double* up, long long n, unsigned long long* count,
                                  hipStream_t s);
hipError_t launch_write_result(const SelArgs& a, uint8_t* mark, int32_t* out_ids, double* out_lo,
                               double* out_up, unsigned long long* rest_bits, int grid, hipStream_t s);
hipError_t launch_all_bounds(const BoundArgs& b, int64_t n, const int32_t* ext_of,
                             double* lower, double* upper, hipStream_t s);
hipError_t launch_init_run(RunScalars* sc, int64_t n, double* sigma, double* sigma_sum,
                           unsigned* xmax32, unsigned long long* xmax64, int max_iter,
                           unsigned* hist, hipStream_t s);

hipError_t launch_prep_rows(const int32_t* ids, long long count, const long long* off, const int* len,
                            long long* blk, int nblocks, long long* sums, long long* totals, RowDesc* desc,
                            SegDesc* segs, HugeRow* huge, RunScalars* sc, const BinBounds& bb, hipStream_t s);

// ---- dynamic update (katz_dynamic.hip) ----------------------------------------
hipError_t launch_scan_ll(const long long* in, long long count, long long* out, long long* sums,
                          long long* total, hipStream_t s);
long long scan_sums_capacity(long long count);
hipError_t launch_slack_caps(const void* rp, int rp64, long long n, int* row_len, int* row_cap,
                             long long* cap_ll, hipStream_t s);
hipError_t launch_copy_rows_to_pool(const void* rp, int rp64, const int32_t* col, long long n, long long nnz,
                                    const long long* row_off, int32_t* pool, hipStream_t s);
// Column ids in range, no self-loop, rows strictly ascending (sc->err |= 1 otherwise).
hipError_t launch_check_rows_strict(const void* rp, int rp64, const int32_t* col, long long n, long long nnz,
                                    RunScalars* sc, hipStream_t s);
// ext_of / int_of: internal <-> caller id maps of a renumbered state (null:
// the state is in caller order); batch pairs and per-row lists are caller ids.
hipError_t launch_batch_exist(const int32_t* a, const int32_t* b, long long n_ins, long long total,
                              const long long* row_off, const int* row_len, const int32_t* pool,
                              const int32_t* ext_of, const int32_t* int_of, int* err, hipStream_t s);
hipError_t launch_map_ids(int32_t* ids, long long count, const int32_t* int_of, hipStream_t s);
hipError_t launch_state_relabel(const RowDesc* desc, long long n, const int* row_cap, int32_t* ext_of,
                               int32_t* int_of, long long* cap_ll, hipStream_t s);
// off_old: row offsets of the old rows by caller id, int64 (off64 = 1) or int32.
hipError_t launch_state_rename_rows(const int32_t* ext_of, const int32_t* int_of, long long n,
                                   const void* off_old, int off64, const int* len_old, const int* cap_old,
                                   const int32_t* pool_old, const long long* off_new, long long used_new,
                                   int* len_new, int* cap_new, int32_t* pool_new, long long* src_of, hipStream_t s);
hipError_t launch_touched_lengths(const int32_t* rows, long long t, const int* delta, const int* row_len,
                                  long long* new_len, uint8_t* mark, hipStream_t s);
hipError_t launch_max_len_after(const int* row_len, const uint8_t* mark, long long n, const long long* new_len,
                                long long t, int* out, hipStream_t s);
hipError_t launch_unmark_rows(const int32_t* rows, long long t, uint8_t* mark, hipStream_t s);
hipError_t launch_merge_rows(const int32_t* rows, long long t, const long long* ins_off, const int* ins_cnt,
                             const int32_t* ins_dst, const long long* del_off, const int* del_cnt,
                             const int32_t* del_dst, const long long* sbase, const long long* row_off,
                             const int* row_len, const int32_t* pool, const int32_t* ext_of, const int32_t* int_of,
                             int32_t* scratch, hipStream_t s);
hipError_t launch_copy_back_rows(const int32_t* rows, long long t, const long long* sbase, const long long* new_len,
                                 const long long* dest_off, const int* dest_cap, const int32_t* scratch,
                                 long long* row_off, int* row_len, int* row_cap, int32_t* pool, hipStream_t s);
// foff: f entries of scratch, sums: scan_sums_capacity(f), total: 1.
// arcs_hint: the host's estimate of the frontier's arcs (0: unknown), which
// only sizes the grid.
hipError_t launch_frontier_expand(const int32_t* frontier, long long f, const long long* row_off, const int* row_len,
                                  const int32_t* pool, int* level_of, int level, int32_t* next, int* next_count,
                                  unsigned long long* next_arcs, long long* foff, long long* sums, long long* total,
                                  unsigned long long arcs_hint, hipStream_t s);
hipError_t launch_set_levels(const int32_t* rows, long long t, int* level_of, int level, hipStream_t s);
hipError_t launch_clear_levels(const int32_t* rows, long long t, int* level_of, hipStream_t s);
hipError_t launch_c_from_history(const int32_t* rows, long long count, double* const* X, int r, double* c,
                                 hipStream_t s);
hipError_t launch_max_of_vector(const double* x, long long n, unsigned long long* out, hipStream_t s);
// FP32 form: c_r = sum_i sigma_i x~_i and the margin recurrence e_i over the
// stored levels, in the order and arithmetic of the walk epilogue.
hipError_t launch_c_from_history_f32(const int32_t* rows, long long count, float* const* X, const double* sigma,
                                     const double* etap, int r, double* c, float* e, hipStream_t s);
// out = max(out, max_v x[v]) as float bits (x >= 0).
hipError_t launch_max_of_vector_f32(const float* x, long long n, unsigned* out, hipStream_t s);

hipError_t launch_reset_flags(RunScalars* sc, hipStream_t s);
hipError_t launch_relabel(const RowDesc* desc, long long n, int32_t* ext_of, int32_t* int_of, long long* coff,
                          IdLen* pmap, long long* len_ll, int* len32, long long* noff, long long* sums,
                          long long* total, hipStream_t s);
hipError_t launch_gather_int(const int32_t* rows, long long t, const int* src, int* out, hipStream_t s);
hipError_t launch_gather_ll(const int32_t* rows, long long t, const long long* src, long long* out, hipStream_t s);
hipError_t launch_min_lower_active(const BoundArgs& b, const int32_t* act, const int* m_ptr,
                                   unsigned long long* min_bits, uint8_t* mark, long long n, hipStream_t s);
hipError_t launch_reactivate_all(const BoundArgs& b, long long n, const unsigned long long* min_bits,
                                 uint8_t* mark, int32_t* out, int* count, hipStream_t s);

hipError_t launch_select_wg(const GraphSel* gsel, int count, const int* r_dev, hipStream_t s);
hipError_t launch_select_wg_one(const GraphSel& one, hipStream_t s);
constexpr int kSmallActive = 1 << 16;   // |M| at or below which one workgroup selects

// ---- batched form (katz_batch.hip) --------------------------------------------
hipError_t launch_batch_prep(const long long* gbase, const void* const* grp, const int* grp64, const long long* gnnz,
                             const long long* gabase, const int32_t* const* gcol, int count, long long total_n,
                             long long total_nnz, int* gid_of, long long* blk, int nblocks, long long* sums,
                             long long* totals, RowDesc* desc, SegDesc* segs, HugeRow* huge, RunScalars* sc,
                             int validate, const BinBounds& bb, hipStream_t s);
hipError_t launch_batch_dmax(const void* const* grp, const int* grp64, const long long* gbase, int count,
                             long long total_n, int* gdmax, hipStream_t s);
hipError_t launch_batch_relabel(const RowDesc* desc, long long total, const long long* gbase, int count,
                                const RunScalars* sc, long long* run_first, long long* run_last,
                                long long* run_start, int32_t* ext_of, int32_t* int_of, long long* coff, IdLen* pmap,
                                long long* len_ll, int* len32, long long* noff, long long* sums, long long* tot,
                                hipStream_t s);
hipError_t launch_batch_rename(const RowDesc* desc, const long long* bin_base, const long long* bin_count,
                               const SegDesc* segs, long long seg_total, const HugeRow* huge, const long long* noff,
                               const int* gid_of, const long long* gbase, const int32_t* const* gcol,
                               const long long* coff, const IdLen* pmap, int32_t* ncol, hipStream_t s);
hipError_t launch_fill_ones(void* x, long long n, int fp32, hipStream_t s);
hipError_t launch_walk_batch(const BatchWalk& a, long long total_blocks, long long max_grid, long long n_huge,
                             hipStream_t s);
hipError_t launch_batch_item_graphs(const BatchWalk& a, long long total_blocks, int* item_g, hipStream_t s);
hipError_t launch_batch_live_items(const BatchWalk& a, long long total_blocks, int* items, int* n_items,
                                   hipStream_t s);
constexpr int kBatchMaxLdsGraphs = 8192;   // per-graph maxima reduced in LDS up to this many graphs
hipError_t launch_batch_advance(int* r_dev, int count, RunScalars* gsc, const unsigned* gxmax32, double* gsigma,
                                double* gsigsum, int* gexp, const double* galpha, const int* gclog2, int stride,
                                int fp32, int* ndone, int* n_items, hipStream_t s);
hipError_t launch_batch_write(const GraphSel* gsel, int count, long long max_n, int32_t* const* out_ids,
                              double* const* out_lo, double* const* out_up, uint8_t* mark,
                              unsigned long long* rest_bits, hipStream_t s);

int bin_of_host(int64_t len, const BinBounds& bb);

// ---- vector kernels of katz_solve (katz_linear.hip) -----------------------------
int linear_reduce_slots();

// ---- reverse graph (katz_transpose.hip) ------------------------------------------
// Device workspace of launch_transpose for a graph of n nodes and nnz arcs.
size_t transpose_scratch_bytes(long long n, long long nnz);
// rt_ptr (n + 1 offsets) and rt_col (nnz ids): the reverse graph of a valid CSR
// (offsets non-decreasing, 0 <= col < n), each reversed row listing its
// sources in ascending order.  scratch: transpose_scratch_bytes(n, nnz) bytes.
hipError_t launch_transpose(const void* rp, int rp64, const int32_t* col, long long n, long long nnz, void* scratch,
                            long long* rt_ptr, int32_t* rt_col, hipStream_t s);
// Sets sc->err when the CSR (rp, col) differs from (rt_ptr, rt_col): with rows
// sorted, a graph equals its transpose exactly when it is symmetric.
hipError_t launch_csr_equal(const void* rp, int rp64, const int32_t* col, const long long* rt_ptr,
                            const int32_t* rt_col, long long n, long long nnz, RunScalars* sc, hipStream_t s);
hipError_t launch_fill_value(double* x, long long n, double v, hipStream_t s);
hipError_t launch_foster_step(const double* y, const double* f, double* f_new, long long n, double* slots,
                              double* out, hipStream_t s);
hipError_t launch_cg_apply(const double* p, const double* y, double* q, long long n, double* slots, double* out,
                           double* scal, hipStream_t s);
hipError_t launch_cg_update(double* z, double* r, const double* p, const double* q, long long n, double* slots,
                            double* out, double* scal, hipStream_t s);
hipError_t launch_cg_direction(double* p, const double* r, const double* scal, long long n, hipStream_t s);
hipError_t launch_write_scores(const double* x, double add, long long n, const int32_t* ext_of, double* out,
                               hipStream_t s);

// ---- dynamic updates in two halves (katz_api.hip) ------------------------------
// How a state reads an update pair (u, v): an undirected edge (arcs u -> v and
// v -> u), a directed arc u -> v, or, in an inbound state (which holds the
// reverse of the caller's graph), the caller's arc u -> v stored as v -> u.
enum PairMode { PAIRS_UNDIRECTED = 0, PAIRS_DIRECTED = 1, PAIRS_REVERSED = 2 };

// The arcs of a batch grouped by the row that stores them.
struct RowGroups {
  std::vector<int32_t> rows;               // touched rows, ascending (caller ids)
  std::vector<long long> ins_off, del_off; // per touched row: first arc in ins_dst / del_dst
  std::vector<int> ins_cnt, del_cnt, delta;
  std::vector<int32_t> ins_dst, del_dst;
};

// A validated batch; prepared on the host without reading the graph, applied
// later to a state of the same n and pair mode.
struct PreparedBatch {
  long long n = 0;
  int mode = PAIRS_UNDIRECTED;
  long long n_ins = 0, n_del = 0;
  std::vector<int32_t> pa;                 // existence-check arcs a -> b: a-ends, then b-ends
  RowGroups fwd;                           // by source row (the state's graph)
  RowGroups rev;                           // directed modes: by target row (the reverse graph)
};
int prepare_batch(long long n, int mode, const int32_t* ins_u, const int32_t* ins_v, long long n_ins,
                  const int32_t* del_u, const int32_t* del_v, long long n_del, PreparedBatch& pb);
int apply_batch(katz_state* st, const PreparedBatch& pb, katz_result* out, hipStream_t s);
int state_pair_mode(const katz_state* st);
long long state_nodes(const katz_state* st);

}  // namespace katz

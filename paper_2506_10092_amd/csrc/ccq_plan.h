// Compiled query plan: the device-side descriptor the kernels read, plus the
// launch entry points implemented in ccq_kernels.hip.  Internal to libccq.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccq {

constexpr int kThreads = 256;          // threads per workgroup (4 wave64)
constexpr int kWaves = kThreads / 64;
constexpr int kRowSpan = 32;           // rows per lane in row mode (one bitmap word)
constexpr int kRowTile = 64 * kRowSpan;   // 2048 rows per wavefront tile (every path)
constexpr int kTileShift = 11;            // log2(kRowTile)
constexpr int kMaxRle = 8;
constexpr int kMaxBp = 4;
constexpr int kMaxIdx = 2;
constexpr int kMaxComp = 2;           // composite columns per query
// the common staged-path instance is compiled for at most this many
// bit-packed columns and accumulators, without MIN / MAX / expression and
// composite code; larger plans take the full instance
constexpr int kSmallBp = 2;
constexpr int kSmallSums = 4;
constexpr int kMaxKeys = 8;
constexpr int kMaxAggs = 8;
constexpr int kLutMaxBits = 14;        // bit-packed columns up to this width get a code table
constexpr int64_t kMaxGroups = int64_t(1) << 27;
constexpr int kLdsTableBytes = 16384;  // group tables up to this size live in LDS
constexpr int64_t kLdsShareGroups = 4096;   // generic row path: tables of at most this many groups stay whole,
constexpr int64_t kLdsShareMin = 1024;      // and larger ones keep at least this many to share the CU
constexpr int kMaxStagedRuns = 1536;  // staged runs per wave slice, all RLE columns together
constexpr int kSegSlots = 64;         // group segments merged per tile in LDS
constexpr int kFastBigBytes = 65536;   // fast row path: largest uint32 count table in dynamic LDS
constexpr int kFastCntWords = 2048;    // fast row path: static LDS counts, (G + 2) * replicas

enum PredKind : int32_t { kPredNone = 0, kPredRange = 1, kPredSet = 2, kPredFalse = 3, kPredIntervals = 4,
                          kPredNotRange = 5 };   // kPredNotRange: v < lo or v >= hi
enum AggKind : int32_t { kAggCount = 0, kAggSumRle = 1, kAggSumBp = 2, kAggSumIdx = 3, kAggExt = 4 };
enum KeySrc : int32_t { kKeyRle = 0, kKeyBp = 1 };

// code table entries (uint16 per code of a bit-packed column)
constexpr uint16_t kLutReject = 0xFFFF;    // code fails the column's predicates
constexpr uint16_t kLutDomain = 0xFFFE;    // code passes but its key is outside [0, card)

struct RleCol {
    const int64_t* ends;
    const void* vals;
    int64_t n_runs;
    int32_t vtype;          // 1 int32, 2 int64
    int32_t pred;           // PredKind
    int64_t lo, hi;         // kPredRange
    const int64_t* set;     // kPredSet: sorted, unique values; kPredIntervals: sorted,
                            // disjoint inclusive pairs (lo0, hi0, lo1, hi1, ...) (device)
    int32_t set_len;        // values, or pairs
    int32_t sum_slot;       // SUM accumulator of this column, or -1
    int32_t key_on;         // 1 if this column is a group key
    int32_t key_shift;
    int64_t key_card;
    int64_t key_stride;
    int32_t stage_base;     // staged paths: first run slot of this column in a wave slice
    int32_t stage_cap;      // and its capacity (>= 64)
    int32_t keep_value;     // staged runs keep the value (a SUM or an expression reads it per row),
                            // not the key's group-id part
    int32_t or_next;        // 1: this column's pass mask is ORed with the next column's (one OR
                            // clause spans consecutive columns); 0: the clause ends here and is ANDed
    int32_t row_clause;     // 1: the clause is the row clause (its mask goes to the row test instead)
};

struct BpCol {
    const uint32_t* packed;
    int64_t base;
    int32_t w;
    int32_t pred;           // PredKind (used when lut == nullptr)
    int64_t lo, hi;
    const int64_t* set;
    int32_t set_len;
    int32_t key;            // key index or -1
    const void* lut;        // device code table (2^w entries of uint8 or uint16) or nullptr
    int32_t lut_u8;         // entries are uint8 (254 = key out of domain, 255 = reject)
    int32_t lut_bytes;      // table size, padded to a multiple of 4
    int64_t n_words;        // words of the stream guaranteed to exist: ceil(rows * w / 32) + 2
    int32_t lut_lds_off;    // byte offset of the code table in dynamic LDS
    int32_t stage_off;      // byte offset of this column's staged words in a wave slice
    int32_t sum_slot;       // SUM accumulator of this column, or -1
    uint32_t code_lo, code_span;   // fast path without code table: codes in [code_lo, code_lo + code_span) pass
    int32_t key_shift;      // key = value >> key_shift when key >= 0 and no code table
    int64_t key_card;
    int64_t key_stride;
    int64_t key_lo;         // no code table: slot = key - key_lo (the reachable keys are contiguous)
    int32_t ones_reject;    // fast path code table: the all-ones code is rejected, so a row the RLE
                            // predicates removed can be sent there by OR-ing its code with all ones
    int32_t pad_ones_;
    // the row clause (an OR over RLE and bit-packed columns): this column's
    // part of it, tested per row on the value (kPredNone: not in it)
    int32_t or_pred;
    int32_t or_set_len;
    int64_t or_lo, or_hi;
    const int64_t* or_set;
    // widths up to kLutMaxBits: that part as one bit per code (device), kept
    // in LDS at or_bits_lds_off (or_bits_words words), instead of testing
    // the value per row
    const uint32_t* or_bits;
    int32_t or_bits_words;
    int32_t or_bits_lds_off;
};

struct IdxCol {
    const void* pos;
    const void* vals;
    int64_t n;
    int32_t ptype, vtype;
    int32_t sum_slot;       // SUM accumulator of this column, or -1
    int32_t pred;           // PredKind on the row's value (0 at rows the column does not list)
    int64_t lo, hi;         // kPredRange
    const int64_t* set;     // kPredSet / kPredIntervals, as for RLE columns (device)
    int32_t set_len;
    int32_t zero_pass;      // 1 when the value 0 passes the predicate
    int32_t or_rcl;         // 1: this mask is an OR clause's Index part, ORed with the clause's RLE
                            // part (the row clause word) before the row mask takes it
    int32_t pad_or_;
};

// A composite column (Section 3.2: RLE + Index, Plain + Index): its base
// part is an ordinary RLE or bit-packed slot without predicates; rows its
// points list take the points' values, and its predicate is tested per row
// on that value (generic row path).
struct CompCol {
    int32_t rle;            // 1: the base part is RLE slot `src`; 0: bit-packed slot `src`
    int32_t src;
    const void* pos;        // points, strictly increasing
    const void* vals;
    int64_t n;
    int32_t ptype, vtype;
    int32_t pred;           // PredKind on the row's value
    int32_t set_len;
    int64_t lo, hi;
    const int64_t* set;
    int32_t lds_off;        // in a wave slice: 64 words of listed rows, then 64 int32 prefixes
    int32_t pad_;
};

struct KeyDesc {
    int32_t src_kind;       // KeySrc
    int32_t src;            // column slot within its kind
    int32_t shift;
    int32_t via_lut;        // slot comes from the bit-packed code table
    int64_t card;
    int64_t radix;          // slots of this key
    int64_t stride;         // mixed-radix weight
    const int64_t* slot_keys;   // via_lut: slot -> key value (device), else nullptr
    const int64_t* dict;        // the key column's dictionary (device): the result reports dict[key]
};

struct AggDesc {
    int32_t kind;           // AggKind
    int32_t src;            // column slot within its kind
    int32_t sum_slot;       // index among the accumulators (-1 for COUNT)
    int32_t fin;            // how the finalize reads the accumulator: kFinValue, kFinMin, kFinMax
};

// MIN and MAX accumulate as an unsigned maximum of an order-preserving
// encoding whose neutral element is 0, so every table starts cleared to 0:
// MIN keeps INT64_MAX - m (larger for smaller m), MAX keeps m ^ 2^63.
enum FinKind : int32_t { kFinValue = 0, kFinMin = 1, kFinMax = 2 };
__host__ __device__ inline uint64_t min_enc(int64_t m) { return (uint64_t)INT64_MAX - (uint64_t)m; }
__host__ __device__ inline int64_t min_dec(uint64_t c) { return (int64_t)((uint64_t)INT64_MAX - c); }
__host__ __device__ inline uint64_t max_enc(int64_t m) { return (uint64_t)m ^ (uint64_t(1) << 63); }
__host__ __device__ inline int64_t max_dec(uint64_t c) { return (int64_t)(c ^ (uint64_t(1) << 63)); }

// An accumulator over a column or a two-column expression, evaluated per
// row on the generic row path (plans with MIN, MAX or an expression).
enum ExtKind : int32_t { kExtNone = 0, kExtSum = 1, kExtMin = 2, kExtMax = 3 };
enum ExtOp : int32_t { kOpNone = 0, kOpAdd = 1, kOpSub = 2, kOpMul = 3 };   // the ABI's CCQ_OP_* values
struct ExtAcc {
    int32_t kind;           // ExtKind
    int32_t op;             // ExtOp
    int32_t a_rle, a_src;   // first operand: RLE (1) or bit-packed (0) column slot
    int32_t b_rle, b_src;   // second operand (op != CCQ_OP_NONE)
};

struct DevPlan;
// the kernel instance's width parameter: the fast row path's width; for
// the staged paths 0 (run mode), -2 (the common generic row path) or -1 (the
// full instance, both modes: composite columns, MIN / MAX / expressions,
// more than kSmallBp bit-packed columns or kSmallSums accumulators)
inline int kernel_w0(const DevPlan& p);

struct DevPlan {
    int64_t row_begin, row_end;
    int64_t tile_rows;      // rows per wavefront tile (64 * span)
    int64_t n_tiles;        // nominal tiles of the window (tiles may end early)
    int32_t span;           // rows per lane
    int32_t row_mode;       // 1 when a bit-packed column is referenced
    int32_t k_rle, n_bp, n_idx, n_keys, n_aggs, n_sums;
    int32_t table_lds;      // 1: per-workgroup LDS table, added to the global one at the end
    int32_t table_c32;      // the LDS table is compact: uint32 counts, int32 sums whose wraps go to
                            // the global table (generic row path)
    int64_t table_lds_groups;   // groups [0, this) have LDS cells ([column][group]); the rest add to
                                // the global table
    uint64_t table_lds_map;     // compact table: LDS column of accumulator `which` (0: COUNT, 1 + k:
                                // SUM slot k) in bits [4 which, 4 which + 4); 15: no LDS column
                                // (an Index SUM, added to the global table)
    int32_t table_lds_cols;     // LDS columns of the compact table
    int32_t any_rle_row;    // row mode: some key or SUM reads an RLE value per row
    int32_t kmax;           // kernel instance: bound on RLE columns (2, 4 or 8)
    int32_t w0;             // kernel instance: width of the fast row path's column (0: none)
    int64_t n_groups;       // product of key radices (1 when ungrouped)
    int32_t run_cap;        // staged runs per wave slice, all RLE columns together
    int32_t lds_dyn_bytes;  // dynamic LDS per workgroup
    int32_t lds_shared_bytes;   // code tables + group table, before the wave slices
    int32_t lds_wave_bytes;     // one wave slice
    int32_t table_lds_off;  // byte offset of the LDS group table
    int32_t off_run_end, off_run_val, off_pts;   // inside a wave slice
    // fast row path: uint32 counts [(G + 2) << rep_shift] in static LDS; in
    // dynamic LDS uint64 code sums [G << rep_shift] and Index sums [n_idx * G]
    int32_t fast_rep_shift, fast_sum_off, fast_isum_off, fast_bytes;
    // fast row path, inside a wave slice: RLE toggle bitmaps (64 words per
    // column); off_pts holds two 64-word lane-mask buffers
    int32_t off_tog;
    int32_t fast_big;       // fast row path with a large table: uint32 counts [G + 2] in dynamic LDS at
                            // fast_sum_off, one replica, slots computed without a code table, Index
                            // sums added to the global table
    // staged paths, inside a wave slice: run-boundary bitmaps and their word
    // prefixes (64 words per RLE column), the lanes' surviving-row words
    int32_t off_bnd, off_bpre, off_pmw;
    int32_t off_rcl;        // staged row mode with a row clause: the RLE part of that clause, one
                            // word per lane (LDS offset in a wave slice), else -1
    // run mode with a global group table: per-wave LDS slots that merge the
    // pieces of one group segment before they reach the table
    int32_t seg_slots, off_slots;
    int32_t n_ext;          // accumulators [0, n_ext) are ExtAcc (MIN, MAX, expressions); 0 otherwise
    int32_t n_comp;         // composite columns (comp[0, n_comp))
    CompCol comp[kMaxComp];
    ExtAcc ext[kMaxAggs];
    RleCol rle[kMaxRle];
    BpCol bp[kMaxBp];
    IdxCol idx[kMaxIdx];
    KeyDesc keys[kMaxKeys];
    AggDesc aggs[kMaxAggs];
};

// ---- batched execution (many plans, one launch sequence)

// A work item: one query and a range of its nominal tiles (relative to the
// query's first tile).
struct BatchItem {
    int32_t query;
    int32_t n_tiles;
    int64_t first_tile;
};

// The items of the queries that share one kernel instance.
struct BatchGroup {
    const BatchItem* items;
    int32_t n_items;
    int32_t kmax, w0;       // kernel instance
    int32_t big;            // fast path with a large table
};

// kernel instance variants besides KMAX: run mode (0, and 5 for plans with
// more than kBatchLdsSplit bytes of LDS), fast row path of width 14 or 20,
// each of those with a large table (1-4), the staged paths' full instance
// (6; w0 = -1: composite columns, MIN / MAX / expressions, wide plans), the
// common generic row path (7; 8 with large LDS, two workgroups per CU; 9
// above kBatchLdsHalf, one workgroup per CU, so such plans do not hold the
// others' launch to one; w0 = -2).  Each instance
// is compiled for its own path, so one path's registers cost no other.
// Variant 5 runs the staged paths' kernel too, for plans that need more
// than kBatchLdsSplit bytes of LDS per workgroup (large group tables in
// LDS), so they do not lower the occupancy of the other staged plans'
// launch.
constexpr int kVariants = 10;
constexpr int kMaxInstances = 3 * kVariants;     // KMAX in {2, 4, 8}
constexpr int kBatchLdsSplit = 48 * 1024;
constexpr int kBatchLdsHalf = 80 * 1024;    // above this, one workgroup per CU
inline int kernel_w0(const DevPlan& p) {
    if (p.w0 > 0) return p.w0;
    if (p.n_comp > 0 || p.n_ext > 0 || p.n_bp > kSmallBp || p.n_sums > kSmallSums) return -1;
    return p.row_mode ? -2 : 0;
}
inline int variant_of(int w0, int big, int lds_bytes) {
    if (w0 == -1) return 6;
    if (w0 == -2) return lds_bytes > kBatchLdsHalf ? 9 : lds_bytes > kBatchLdsSplit ? 8 : 7;
    return w0 == 0 ? (lds_bytes > kBatchLdsSplit ? 5 : 0) : (w0 == 14 ? 1 : 2) + (big ? 2 : 0);
}
inline int variant_w0(int v) {
    return v == 6 ? -1 : (v == 7 || v == 8 || v == 9) ? -2 : v == 0 || v == 5 ? 0 : (v == 1 || v == 3) ? 14 : 20;
}
inline int variant_big(int v) { return v == 3 || v == 4 ? 1 : 0; }

// Where each query's result goes.
struct BatchOut {
    int64_t *keys, *counts, *aggs, *n_groups;
    int32_t* status;
};

// Each query owns a region of the workspace laid out like a single query's
// workspace (status header, group table, finalize scan) at byte offset
// region[q]; the first region_clear[q] bytes are cleared before the launch.
// counters: one int32 item counter per group (cleared with the regions).
struct BatchDev {
    const DevPlan* const* plans;     // [n] device plans
    const int64_t* region;           // [n] byte offset of query q's region in the workspace
    const int64_t* region_clear;     // [n] bytes of the region to clear
    const BatchOut* outs;            // [n]
    int32_t* counters;               // [kMaxInstances] device item counters
    BatchGroup groups[kMaxInstances];
    int32_t n_groups_used;
    int32_t n;
};

// Launch a whole batch on `stream`: clear every query's region and the
// counters, one persistent launch per kernel instance, one finalize
// workgroup per query, then the multi-block finalize for the queries listed
// in big (group tables over kBatchFinMaxGroups ids).  Host arrays:
// plans_host (host copies), plans_dev (device plan pointers), region, outs.
// ev_begin / ev_end (or null): recorded right before the first and after
// the last persistent launch.
hipError_t launch_batch(const BatchDev& host, const BatchDev* dev, const DevPlan* const* plans_host,
                        const DevPlan* const* plans_dev, const int64_t* region, const BatchOut* outs,
                        unsigned char* ws, const int* group_grid, const int* group_lds, const int32_t* big,
                        int32_t n_big, hipStream_t stream, hipEvent_t ev_begin = nullptr,
                        hipEvent_t ev_end = nullptr, int32_t fin_grid = 0);

// Persistent-grid size and dynamic LDS of a batch kernel instance.
int batch_grid_limit(int kmax, int w0, int big, int lds_bytes, int cus);

// Largest work item, in 2048-row tiles: one workgroup counts an item's rows
// in uint32 LDS counters, so an item stays below 2^31 rows.
constexpr int32_t kMaxTilesPerItem = int32_t(1) << 19;

// Largest group count the single-workgroup batched finalize handles.
constexpr int64_t kBatchFinMaxGroups = int64_t(1) << 20;

// Workspace layout (device, 256-byte aligned pieces):
//   [0, 256)   header: int32 status, int32 spare
//   table      (1 + n_sums) * n_groups int64: counts, then each SUM
//   scan       finalize block counts
struct WsLayout {
    size_t table_off, scan_off, total;
    int64_t scan_blocks;
};

WsLayout workspace_layout(const DevPlan& p);

// Launch the whole query on `stream`: prepare (clear), fused
// filter/align/aggregate, finalize.  `dp` is the device copy of `p`.
hipError_t launch_query(const DevPlan& p, const DevPlan* dp, void* ws, hipStream_t stream, int64_t* out_keys,
                        int64_t* out_counts, int64_t* out_aggs, int64_t* out_n_groups, int32_t* out_status,
                        int grid_fused, hipEvent_t ev_begin, hipEvent_t ev_end);

// Size of the fixed device scratch that ccq_execute_noalloc uses as the
// workspace, and the lookup of its address on the current device.
constexpr size_t kScratchBytes = size_t(32) << 20;
hipError_t scratch_address(void** out);

// Kernel instances (ccq_inst.hip, one object per RLE-column bound 2 / 4 / 8):
// w0 = 0 for the staged paths, 14 or 20 for the fast row path; big = that
// path with a large table.
typedef void (*FusedFn)(const DevPlan*, int64_t*, int32_t*, int64_t);
typedef void (*BatchFn)(const BatchDev*, int32_t, unsigned char*);
FusedFn fused_kernel_k2(int w0, bool big);
FusedFn fused_kernel_k4(int w0, bool big);
FusedFn fused_kernel_k8(int w0, bool big);
BatchFn batch_kernel_k2(int w0, bool big);
BatchFn batch_kernel_k4(int w0, bool big);
BatchFn batch_kernel_k8(int w0, bool big);

// Device validation of one column; writes a nonzero flag on failure.
hipError_t launch_validate_rle(const int64_t* ends, int64_t n, int64_t n_rows, int32_t* flag, hipStream_t s);
hipError_t launch_validate_idx(const void* pos, int32_t ptype, int64_t n, int64_t n_rows, int32_t* flag,
                               hipStream_t s);

// Persistent-grid size for the fused kernel with the plan's LDS use.
int fused_grid_limit(const DevPlan& p, int cus);

// Static LDS of a k_fused / k_batch instance (s_lut, s_cnt, s_item), with
// slack for alignment: a plan's dynamic LDS must stay within the
// workgroup's LDS minus this.
constexpr int kernel_static_lds(int w0, int big) {
    return ((w0 > 0 && w0 <= kLutMaxBits && !big) ? (1 << w0) + 16 : 16) + 4 * ((w0 > 0 && !big) ? kFastCntWords : 4) +
           4 + 256;
}

// Bit widths that have a fast row-mode kernel instance.
bool fast_row_width(int w);

}  // namespace ccq

/*
 * ccq.h -- filter / group-by / aggregate queries that run directly on
 * lightweight-compressed columns on an MI355X (gfx950) GPU.
 *
 * The operation follows the paper's statement of the problem
 * (arXiv 2506.10092, "GPU Acceleration of SQL Analytics on Compressed Data"):
 *   - columns arrive encoded (Section 3.1: Plain, RLE, Index; Section 3.2:
 *     bit-width reduction around a global reference value; dictionary codes
 *     are plain integer codes, Section 2.1);
 *   - a query is a conjunction of selection predicates, each possibly negated
 *     (Sections 5.1, 5.3 and 6),
 *     a list of group-by keys and SUM / COUNT(*) aggregates (Section 7);
 *   - the answer is the exact aggregate per non-empty group, in ascending key
 *     order (torch.unique order, Section 2.2).  RLE runs contribute
 *     value * run length to SUM and run length to COUNT (Section 7,
 *     "Aggregating Phase"); runs of several RLE columns are first aligned to
 *     their common refinement (Section 6, Alignment; Algorithm 1).
 *
 * Conventions (readings of the paper, see the design notes):
 *   - an RLE column stores values[i] and an EXCLUSIVE run end run_ends[i]:
 *     run i covers rows [run_ends[i-1], run_ends[i]) (run_ends[-1] = 0), i.e.
 *     the paper's inclusive end plus one; base columns have no gaps;
 *   - an Index column lists (position, value) pairs; rows it does not list
 *     hold the value 0 (for SUM and for predicates on the column);
 *   - a bit-packed column stores row r's code in bits [r*w, r*w + w) of an
 *     LSB-first stream of little-endian uint32 words; value = base + code;
 *   - RANGE predicates are half open, lo <= v < hi; IN has set semantics;
 *   - a group key is v >> shift (arithmetic) and must lie in [0, card);
 *   - all arithmetic is exact int64 (sums wrap only where int64 overflows,
 *     which callers must rule out).
 *
 * Memory: every column buffer, workspace and result buffer is DEVICE memory
 * owned by the caller (e.g. torch tensors); the library borrows column
 * buffers for the lifetime of the table and plans built on them and never
 * writes to them.  Host descriptors and IN-lists are copied at create time.
 * The library allocates device memory only in ccq_plan_create (the compiled
 * plan) -- never in ccq_execute.
 *
 * Errors: every call returns CCQ_OK (0) or a negative ccq_status; a
 * thread-local message is available from ccq_last_error().  Errors that
 * depend on data values (a group key outside its domain) are written to the
 * result's device status word by the kernels and are readable after the
 * stream is synchronised.  No C++ exception crosses this interface.
 *
 * Threading: a context, table or plan may be used from several host threads;
 * a plan is immutable after creation and may run concurrently on different
 * streams as long as each call has its own workspace and result buffers.
 */
#ifndef CCQ_H
#define CCQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CCQ_ABI_VERSION 8

typedef int32_t ccq_status;
enum {
    CCQ_OK = 0,
    CCQ_E_INVALID = -1,      /* malformed argument, descriptor or plan */
    CCQ_E_UNSUPPORTED = -2,  /* well formed, but outside what the kernels implement */
    CCQ_E_CAPACITY = -3,     /* workspace or result buffer too small */
    CCQ_E_KEY_DOMAIN = -4,   /* (device status) a group key fell outside [0, card) */
    CCQ_E_HIP = -5,          /* HIP runtime error (message has the detail) */
    CCQ_E_BUDGET = -6,       /* server: the query does not fit the HBM budget */
    CCQ_E_BUSY = -7,         /* server: queue full */
    CCQ_E_NOMEM = -8         /* host or device allocation failed */
};

typedef struct ccq_context ccq_context;
typedef struct ccq_table ccq_table;
typedef struct ccq_plan ccq_plan;

/* ---- encodings (Section 3.1 Basic Encodings; Section 3.2 bit widths and
 * composite encodings) ----
 * CCQ_RLE_INDEX (Section 3.2, RLE + Index): pure runs plus Index points on
 * the rows no pure run covers.  The RLE part is values / run_ends /
 * n_entries with run_ends as for CCQ_RLE (strictly increasing, last ==
 * rows): run i stands for the rows of [run_ends[i-1], run_ends[i]) (0 for
 * i = 0) that no point lists, so a pure run's start is implicit.  From
 * runs given with starts and ends (ccq_plain_to_rle_index), keep the ends
 * and set the last one to the row count; a column of points only takes one
 * run over every row, whose value is never read.
 * CCQ_PLAIN_INDEX (Section 3.2, Plain + Index): a BITPACKED column (packed,
 * bit_width, base) whose rows listed as points take the points' values; the
 * codes at those rows are never read.
 * Both composites list their points in positions (position_type) and
 * point_values (value_type), n_points of them, positions strictly increasing
 * in [0, rows).  A query may name at most two composite columns, in
 * predicates (alone in their OR clauses), SUM, MIN, MAX and expression
 * operands, not in group keys; such queries take the generic row path. */
enum { CCQ_RLE = 1, CCQ_INDEX = 2, CCQ_BITPACKED = 3, CCQ_RLE_INDEX = 4, CCQ_PLAIN_INDEX = 5 };
enum { CCQ_I32 = 1, CCQ_I64 = 2 };

typedef struct {
    int32_t encoding;          /* CCQ_RLE, CCQ_INDEX, CCQ_BITPACKED, CCQ_RLE_INDEX or CCQ_PLAIN_INDEX */
    int32_t value_type;        /* RLE, INDEX and the composites: CCQ_I32 or CCQ_I64 */
    int64_t n_entries;         /* RLE, RLE_INDEX: runs; INDEX: listed points; BITPACKED, PLAIN_INDEX:
                                  rows (== table rows) */
    const void* values;        /* RLE, INDEX: device value_type[n_entries] */
    const int64_t* run_ends;   /* RLE: device int64[n_entries], exclusive, strictly
                                  increasing, first > 0, last == table rows */
    const void* positions;     /* INDEX: device position_type[n_entries], strictly
                                  increasing in [0, table rows) */
    const uint32_t* packed;    /* BITPACKED: device stream of >= ceil(rows*w/32) + 2 words */
    int32_t bit_width;         /* BITPACKED: 1..32 */
    int32_t position_type;     /* INDEX: CCQ_I32 or CCQ_I64 */
    int64_t base;              /* BITPACKED: value = base + code */
    const int64_t* dict_values;  /* BITPACKED, optional (NULL: none): device int64[dict_size], the
                                  dictionary of a dictionary-encoded column (Section 2.1).  Predicates,
                                  keys and the row order see the code value (base + code); a group key on
                                  this column reports dict_values[key] in the result instead of the key.
                                  Such a key needs shift 0 and card <= dict_size; SUM over the column is
                                  CCQ_E_UNSUPPORTED.  Borrowed like the other column buffers. */
    int64_t dict_size;         /* entries of dict_values (>= 1 when dict_values is set, else 0) */
    const void* point_values;  /* RLE_INDEX, PLAIN_INDEX: device value_type[n_points], the Index part's
                                  values (positions in `positions`) */
    int64_t n_points;          /* RLE_INDEX, PLAIN_INDEX: listed points (>= 0); 0 for the other encodings */
} ccq_column_desc;

/* ---- query (Sections 5-7) ----
 * CCQ_NOT_RANGE and CCQ_NOT_IN hold where CCQ_RANGE and CCQ_IN fail: the
 * complement of the predicate's mask (Section 5.3, NOT; Algorithms 7 and 8
 * complement RLE and Index masks).
 *
 * The filter is a conjunction of clauses.  A predicate with clause == 0 is a
 * clause of its own; predicates sharing a clause id k > 0 form one clause,
 * their OR (Section 5.2, OR of masks: range_union for RLE masks, a merge of
 * positions for Index masks).  With NOT this expresses any filter over the
 * predicates (De Morgan; the composite-mask rules of Section 5).  Predicates
 * on one column fold into one list of value intervals: AND intersects, OR
 * unites, NOT complements.  An OR clause over one column takes any
 * encoding.  An OR clause over several columns names RLE columns, except
 * that one clause per query may also name bit-packed columns (Table 4, RLE
 * mask OR Plain mask) or, instead, exactly one Index column (Table 4, RLE
 * mask OR Index mask; the column holds 0 at its unlisted rows).  Such an
 * Index column takes one of the query's two Index column slots beyond any
 * it takes for its other predicates or SUMs.  At most 8 RLE column uses per
 * query, counting each column once for the clause-0 predicates, keys and
 * SUMs and once per clause over several columns that names it.  Otherwise
 * CCQ_E_UNSUPPORTED. */
enum { CCQ_RANGE = 1, CCQ_IN = 2, CCQ_NOT_RANGE = 3, CCQ_NOT_IN = 4 };
typedef struct {
    int32_t col;               /* column index in the table */
    int32_t op;                /* CCQ_RANGE: lo <= v < hi;  CCQ_IN: v in in_list;
                                  CCQ_NOT_RANGE / CCQ_NOT_IN: the negations */
    int64_t lo, hi;
    const int64_t* in_list;    /* CCQ_IN, CCQ_NOT_IN: HOST array, copied by ccq_plan_create */
    int64_t in_len;
    int32_t clause;            /* 0: ANDed on its own; k > 0: ORed with the other predicates of clause k,
                                  the clause ANDed; must be >= 0 */
    int32_t pad_;              /* ignored */
} ccq_pred;

typedef struct {
    int32_t col;               /* RLE or BITPACKED column */
    int32_t shift;             /* key = v >> shift, 0..62 */
    int64_t card;              /* the key must lie in [0, card) */
} ccq_key;

/* Aggregates (Section 7.2, aggregating phase): COUNT(*), SUM, MIN, MAX of a
 * column, or of the row-wise sum, difference or product of two columns
 * (Section 6: arithmetic on columns after aligning their runs).  Arithmetic
 * is int64 and wraps (equal to the exact value whenever that fits in int64).
 * For an ungrouped query with no qualifying row every aggregate is 0.
 * AVG, STD and VAR are post-processing of COUNT, SUM(x) and SUM(x * x)
 * (ccq_avg_var).  MIN, MAX and the two-column forms take RLE and BITPACKED
 * columns (an INDEX column: CCQ_E_UNSUPPORTED); SUM of one column takes any
 * encoding. */
enum { CCQ_COUNT_STAR = 1, CCQ_SUM = 2, CCQ_MIN = 3, CCQ_MAX = 4 };
enum { CCQ_OP_NONE = 0, CCQ_OP_ADD = 1, CCQ_OP_SUB = 2, CCQ_OP_MUL = 3 };
typedef struct {
    int32_t func;              /* CCQ_COUNT_STAR, CCQ_SUM, CCQ_MIN or CCQ_MAX */
    int32_t col;               /* the column (ignored for COUNT(*)) */
    int32_t op;                /* CCQ_OP_NONE: the column; else col op col2, row by row */
    int32_t col2;              /* second column when op != CCQ_OP_NONE */
} ccq_agg;

typedef struct {
    const ccq_pred* preds;  int32_t n_preds;   /* conjunction of clauses (see ccq_pred.clause) */
    const ccq_key* keys;    int32_t n_keys;    /* GROUP BY, first key most significant */
    const ccq_agg* aggs;    int32_t n_aggs;
    int64_t row_begin, row_end;                /* logical window [row_begin, row_end) */
} ccq_query_desc;

/* Result buffers (DEVICE memory, caller owned).  After the stream is
 * synchronised: *n_groups rows are valid; row g has keys[g*n_keys + k],
 * counts[g] (= COUNT(*) of the group) and aggs[g*n_aggs + a] (COUNT(*)
 * aggregates repeat counts[g]).  Grouped queries list only groups with
 * count > 0, in ascending key order.  An ungrouped query always yields one
 * row (count 0 and sums 0 when nothing qualifies).  *status is CCQ_OK or a
 * data-dependent error (CCQ_E_KEY_DOMAIN), in which case the rows are not
 * meaningful.  capacity must be >= the plan's max_groups (ccq_plan_info). */
typedef struct {
    int64_t* keys;
    int64_t* counts;
    int64_t* aggs;
    int64_t* n_groups;
    int32_t* status;
    int64_t capacity;
} ccq_result;

/* ---- calls ---- */

/* Message of the last failed call on this thread ("" if none). */
const char* ccq_last_error(void);
int32_t ccq_abi_version(void);

/* A context binds a HIP device (the device is made current on each call).
 * device == CCQ_HOST_ONLY makes a context without a device: tables can be
 * described and plans checked (ccq_plan_check), nothing can run. */
#define CCQ_HOST_ONLY (-1)
ccq_status ccq_context_create(int32_t device, ccq_context** out);
void ccq_context_destroy(ccq_context* ctx);              /* NULL-safe */

/* A table: n_rows logical rows and n_cols encoded columns.  Host-side checks
 * only (counts, widths, pointer presence); see ccq_table_validate for the
 * O(data) device check. */
ccq_status ccq_table_create(ccq_context* ctx, int64_t n_rows, const ccq_column_desc* cols, int32_t n_cols,
                            ccq_table** out);
void ccq_table_destroy(ccq_table* t);                    /* NULL-safe; plans keep their own copy */

/* Check on the device that run ends are strictly increasing with the last
 * equal to n_rows and that positions are strictly increasing in range.
 * Synchronises `stream`; returns CCQ_OK or CCQ_E_INVALID (naming the first
 * bad column).  It only reads inside each column's arrays.
 * Precondition of every execution: the kernels trust run ends and positions
 * (they index LDS tiles and packed words by them), so running a plan on a
 * table whose columns break these rules is undefined behaviour (wrong
 * results or faulting accesses).  Callers that did not build the columns
 * themselves should validate the table once, before its first execution. */
ccq_status ccq_table_validate(ccq_table* t, void* stream);

/* Compile a query against a table: validates the query, folds predicates
 * per column, builds code lookup tables, chooses tiles and allocates the
 * plan's device descriptor.  CCQ_E_UNSUPPORTED for query shapes the kernels
 * do not implement (keys on INDEX columns, OR clauses outside the forms
 * above, more than 8 RLE column uses or 4 bit-packed columns, more than 2^27
 * key combinations). */
ccq_status ccq_plan_create(const ccq_table* t, const ccq_query_desc* q, ccq_plan** out);
void ccq_plan_destroy(ccq_plan* p);                      /* NULL-safe */

/* Validate and compile a query without allocating anything: the same
 * checks and status codes as ccq_plan_create, plus the result bound and the
 * workspace size a plan for it would report. */
ccq_status ccq_plan_check(const ccq_table* t, const ccq_query_desc* q, int64_t* max_groups,
                          size_t* workspace_bytes);

/* Upper bound on result rows and the workspace size ccq_execute needs. */
ccq_status ccq_plan_info(const ccq_plan* p, int64_t* max_groups, size_t* workspace_bytes);

/* Run one query on `stream` (a hipStream_t, or NULL for the null stream).
 * Asynchronous: returns after enqueueing.  workspace: device buffer of at
 * least workspace_bytes, 256-byte aligned, not shared with a concurrent call.
 * Result rows are written as described at ccq_result. */
ccq_status ccq_execute(const ccq_plan* p, void* workspace, size_t workspace_bytes, void* stream,
                       const ccq_result* result);

/* Options for ccq_execute_ex.  fused_begin / fused_end: hipEvent_t handles
 * (or NULL) recorded on `stream` immediately before and after the fused
 * filter / align / aggregate kernel, so a caller can time that kernel alone
 * with hipEventElapsedTime. */
typedef struct {
    void* fused_begin;
    void* fused_end;
} ccq_exec_opts;

/* ccq_execute with options (opts may be NULL). */
ccq_status ccq_execute_ex(const ccq_plan* p, void* workspace, size_t workspace_bytes, void* stream,
                          const ccq_result* result, const ccq_exec_opts* opts);

/* ccq_execute without a caller workspace, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid allocation).  The query's workspace is a fixed device array of
 * CCQ_NOALLOC_WORKSPACE_BYTES that the library holds on every device it runs
 * on until the process ends (its address is looked up when the context is
 * created).  Nothing is allocated or freed: no hipMalloc / hipFree, no
 * allocating library call.  The launch sequence clears what must start at
 * zero (status header, group table) itself.  Every call on one device shares
 * that array, so calls whose execution overlaps on one device (other streams,
 * other threads, other contexts of the device) race and give wrong results;
 * serialise them.  Returns CCQ_E_CAPACITY when the plan's workspace
 * (ccq_plan_info) exceeds CCQ_NOALLOC_WORKSPACE_BYTES, and otherwise the
 * codes of ccq_execute; results are identical to ccq_execute's. */
#define CCQ_NOALLOC_WORKSPACE_BYTES ((size_t)32 << 20)
ccq_status ccq_execute_noalloc(const ccq_plan* p, void* stream, const ccq_result* result);

/* AVG and population VAR per result row from COUNT, SUM(x) and SUM(x * x)
 * (Section 7.2: computed after SUM and COUNT): each exact int64 is rounded
 * to the nearest double, then avg = s / n and var = (ss - s * s / n) / n in
 * IEEE double arithmetic, in that order (0 and 0 when n = 0).  Host arrays of
 * n_rows entries; returns CCQ_E_INVALID for NULL arrays or n_rows < 0. */
ccq_status ccq_avg_var(const int64_t* count, const int64_t* sum, const int64_t* sum_sq, int64_t n_rows, double* avg,
                       double* var);

/* ---- encoding Plain data on the device (Table 1: plain_to_rle,
 * plain_to_rle+index, plain_to_plain+index) and choosing an encoding
 * (Section 9, the evaluation's encoding heuristics) ----
 *
 * Input: a device array of n_rows values (value_type CCQ_I32 or CCQ_I64), in
 * row order.  Every call needs a device workspace of at least
 * ccq_encode_workspace_bytes(n_rows) bytes, 256-byte aligned, not shared with
 * a concurrent call.  Each call enqueues its kernels on `stream` and
 * synchronises it (the output sizes are read back before anything is
 * written); outputs are device arrays owned by the caller.  Errors:
 * CCQ_E_INVALID (arguments), CCQ_E_CAPACITY (workspace or an output too
 * small: nothing is written, the sizes needed are still returned),
 * CCQ_E_HIP. */
enum { CCQ_CHOOSE_PLAIN = 1, CCQ_CHOOSE_RLE = 2, CCQ_CHOOSE_RLE_INDEX = 3, CCQ_CHOOSE_PLAIN_INDEX = 4 };

typedef struct {
    int64_t n_rows;
    int64_t runs;            /* maximal runs of equal values */
    int64_t single_runs;     /* of them, runs of one row */
    int64_t min_value, max_value;
    int64_t lo_cut, hi_cut;  /* the values at sorted ranks floor(n/20) and n - 1 - floor(n/20)
                                (the top and bottom 5% cut) */
    int32_t choice;          /* CCQ_CHOOSE_*: under 1e6 rows Plain; else RLE when
                                n * sizeof(value) / (runs * (sizeof(value) + 16)) > 20 (a run as
                                value, start, end); else RLE+Index when there are single-row runs
                                and (n - single runs) * sizeof(value) / (longer runs *
                                (sizeof(value) + 16)) > 20; else Plain+Index when the cut range
                                needs fewer bits than the full range; else Plain (RLE when even
                                Plain would need more than 32 bits) */
    int32_t bit_width;       /* PLAIN, PLAIN_INDEX: code width (1..32); 0 for the other choices */
    int64_t base;            /* PLAIN, PLAIN_INDEX: value = base + code (PLAIN: the minimum;
                                PLAIN_INDEX: centered, the cut range's midpoint rounded up minus
                                2^(bit_width - 1), at least INT64_MIN) */
    int64_t rle_runs;        /* RLE: runs; RLE_INDEX: runs of two or more rows */
    int64_t index_points;    /* RLE_INDEX: single-row runs; PLAIN_INDEX: rows outside
                                [base, base + 2^bit_width) */
} ccq_encoding_choice;

size_t ccq_encode_workspace_bytes(int64_t n_rows);

/* Column statistics and the encoding the heuristics choose. */
ccq_status ccq_encode_choose(ccq_context* ctx, const void* values, int32_t value_type, int64_t n_rows, void* ws,
                             size_t ws_bytes, void* stream, ccq_encoding_choice* out);

/* Plain -> RLE: maximal runs.  run_values: value_type[capacity], run_ends:
 * int64[capacity] (exclusive ends; the form ccq_table_create takes);
 * *n_runs (host) receives the number of runs. */
ccq_status ccq_plain_to_rle(ccq_context* ctx, const void* values, int32_t value_type, int64_t n_rows, void* ws,
                            size_t ws_bytes, void* stream, void* run_values, int64_t* run_ends, int64_t capacity,
                            int64_t* n_runs);

/* Plain -> RLE+Index (Section 3.2, composite encodings): runs of two or
 * more rows as RLE (values, starts, exclusive ends; gaps where points are),
 * rows whose run is a single row as Index points (int64 positions,
 * value_type values).  Runs and points are disjoint and cover every row. */
ccq_status ccq_plain_to_rle_index(ccq_context* ctx, const void* values, int32_t value_type, int64_t n_rows,
                                  void* ws, size_t ws_bytes, void* stream, void* run_values, int64_t* run_starts,
                                  int64_t* run_ends, int64_t run_capacity, int64_t* idx_positions, void* idx_values,
                                  int64_t idx_capacity, int64_t* n_runs, int64_t* n_points);

/* Plain -> Plain+Index (Section 3.2): codes value - base of bit_width bits,
 * packed as a BITPACKED column (>= ceil(n*w/32) + 2 words; rows outside
 * [base, base + 2^bit_width) hold code 0 there) and those rows as Index
 * points (int64 positions, value_type values). */
ccq_status ccq_plain_to_plain_index(ccq_context* ctx, const void* values, int32_t value_type, int64_t n_rows,
                                    int32_t bit_width, int64_t base, void* ws, size_t ws_bytes, void* stream,
                                    uint32_t* packed, int64_t packed_words, int64_t* idx_positions, void* idx_values,
                                    int64_t idx_capacity, int64_t* n_points);

/* ---- joins on encoded columns (Section 8: Get Join Index, Apply Join Index) ----
 *
 * An equi-join of column left_col of `left` (rows [left_begin, left_end))
 * with column right_col of `right` (rows [right_begin, right_end)), on the
 * columns' integer values (a bit-packed column's base + code; a dictionary
 * column joins on its codes).  The join works on entries: an RLE run (its
 * value and its rows, clipped to the window), a listed point of an Index
 * column (rows an Index column does not list take no part), or one row of a
 * bit-packed column.  Each pair of equal-valued entries gives one block, the
 * cross product of the two entries' row ranges: an RLE side keeps its join
 * index as row ranges, the other encodings as single rows (Table 6).  The
 * join's row pairs are the blocks' pairs, block by block with the left row
 * outer; blocks of one left entry are adjacent and left entries come in row
 * order, but the order of the blocks within one left entry is unspecified
 * (the Join Index is unsorted).
 *
 * Both tables need device contexts on one device.  Workspace: device memory
 * of ccq_join_workspace_bytes(...) bytes (same arguments), 256-byte
 * aligned, not shared with a concurrent call.  ccq_join_index enqueues its
 * kernels on `stream` and synchronises it twice (entry counts, then the
 * number of blocks); `blocks` is a device array of `capacity` blocks owned by
 * the caller.  *n_blocks and *n_pairs (host) receive the number of blocks and
 * of row pairs (the join's output rows; below 2^63 assumed) also when the
 * capacity is too small (CCQ_E_CAPACITY, nothing written).  Errors:
 * CCQ_E_INVALID (NULL pointers, column or window out of range, host-only
 * context, misaligned workspace), CCQ_E_CAPACITY, CCQ_E_HIP.  Run ends and
 * positions must satisfy ccq_table_validate. */
typedef struct {
    int64_t left_start, left_len;    /* rows [left_start, left_start + left_len) of the left table */
    int64_t right_start, right_len;  /* rows [right_start, right_start + right_len) of the right table */
} ccq_join_block;

size_t ccq_join_workspace_bytes(const ccq_table* left, int32_t left_col, int64_t left_begin, int64_t left_end,
                                const ccq_table* right, int32_t right_col, int64_t right_begin, int64_t right_end);
ccq_status ccq_join_index(const ccq_table* left, int32_t left_col, int64_t left_begin, int64_t left_end,
                          const ccq_table* right, int32_t right_col, int64_t right_begin, int64_t right_end, void* ws,
                          size_t ws_bytes, void* stream, ccq_join_block* blocks, int64_t capacity, int64_t* n_blocks,
                          int64_t* n_pairs);

/* Apply Join Index: out[p] = the value of column `col` of table t at the
 * side's row of the join's p-th pair (side 0: left rows, 1: right rows), in
 * the pair order above; an Index column holds 0 at rows it does not list;
 * a bit-packed column gives base + code.  blocks: device array of n_blocks
 * (from ccq_join_index over t as that side, or any blocks whose side rows
 * lie in t, with pairs per block below 2^63).  Workspace: device memory of
 * ccq_join_apply_workspace_bytes(n_blocks, n_pairs) bytes, 256-byte aligned,
 * n_pairs the blocks' pairs (ccq_join_index reports it; a call with a
 * workspace for n_pairs = 0 and capacity 0 reports it in *n_out with
 * CCQ_E_CAPACITY).
 * Synchronises `stream` once (the number of pairs), then enqueues the gather;
 * out: device int64[capacity]; *n_out (host) receives the number of pairs
 * also on CCQ_E_CAPACITY (nothing written).  CCQ_E_INVALID for a block with a
 * negative length or side rows outside the table (checked on the device
 * before anything is written). */
size_t ccq_join_apply_workspace_bytes(int64_t n_blocks, int64_t n_pairs);
ccq_status ccq_join_apply(const ccq_table* t, int32_t col, const ccq_join_block* blocks, int64_t n_blocks, int32_t side,
                          void* ws, size_t ws_bytes, void* stream, int64_t* out, int64_t capacity, int64_t* n_out);

/* ---- batched execution: many queries, one launch sequence ----
 *
 * A batch runs n compiled plans (over any tables of one device) together:
 * one clear, one persistent launch per kernel variant in which workgroups
 * take (query, range of tiles) work items from a device counter, and one
 * finalize for all queries.  Each query's answer is exactly what
 * ccq_execute gives for its plan.  Result buffers are fixed at creation;
 * the workspace is passed per execution (ccq_batch_info gives its size). */
typedef struct ccq_batch ccq_batch;

typedef struct {
    int32_t tiles_per_item;    /* tiles per work item (0: default 64); a tuning knob, no effect on results */
    int32_t use_graph;         /* 1: capture the launch sequence as a hipGraph on the first execution with a
                                  given (workspace, stream) and replay it afterwards (needs a non-NULL stream) */
} ccq_batch_opts;

ccq_status ccq_batch_create(ccq_context* ctx, const ccq_plan* const* plans, int32_t n, const ccq_result* results,
                            const ccq_batch_opts* opts, ccq_batch** out);
void ccq_batch_destroy(ccq_batch* b);                    /* NULL-safe */

/* Workspace bytes the batch needs and the number of work items. */
ccq_status ccq_batch_info(const ccq_batch* b, size_t* workspace_bytes, int64_t* n_items);

/* Change the work-item size (rebuilds the item lists; drops a captured graph). */
ccq_status ccq_batch_set_tiles_per_item(ccq_batch* b, int32_t tiles_per_item);

/* Run every query of the batch on `stream`; asynchronous like ccq_execute. */
ccq_status ccq_batch_execute(ccq_batch* b, void* workspace, size_t workspace_bytes, void* stream);

/* ccq_batch_execute with options (opts may be NULL).  With events set, the
 * fused_begin / fused_end events of ccq_exec_opts are recorded on `stream`
 * right before the first and after the last persistent launch of the batch,
 * so those launches can be timed together; such an execution is launched
 * directly, never replayed from the captured graph. */
ccq_status ccq_batch_execute_ex(ccq_batch* b, void* workspace, size_t workspace_bytes, void* stream,
                                const ccq_exec_opts* opts);

/* Time each candidate work-item size (reps executions each, after one warm-up;
 * synchronises `stream`), keep the fastest by median, report it and its time.
 * The result is kept in the context's tuning cache, keyed by the batch's
 * shape: the device's architecture and CU count, the candidate list, and per
 * query its kernel instance, nominal tiles, group count, accumulators and
 * LDS bytes.  A batch whose key is cached (from an earlier autotune or a
 * loaded cache file) takes the cached size and time without executing
 * anything. */
ccq_status ccq_batch_autotune(ccq_batch* b, void* workspace, size_t workspace_bytes, void* stream,
                              const int32_t* candidates, int32_t n_candidates, int32_t reps, int32_t* best,
                              float* best_ms);

/* The tuning cache as a text file: a header line, then one line per entry
 * (the key in hex, the work-item size, the median time in ms).
 * ccq_tune_cache_load merges a file into the context's cache (a missing file
 * loads nothing and succeeds); ccq_tune_cache_save writes the whole cache to
 * `path` (through a temporary file renamed over it).  Host paths; *n_entries
 * (may be NULL) receives the entries read or written.  CCQ_E_INVALID for a
 * NULL context or path, a file that is not a tuning cache (nothing merged),
 * or an I/O error (the message carries the system's).  Safe to call while
 * other threads autotune batches of the same context. */
ccq_status ccq_tune_cache_load(ccq_context* ctx, const char* path, int64_t* n_entries);
ccq_status ccq_tune_cache_save(ccq_context* ctx, const char* path, int64_t* n_entries);

/* ---- serving: continuous batching under an HBM budget ----
 *
 * A server owns a device arena of hbm_budget_bytes (allocated once, at
 * creation) from which every admitted query gets its workspace, and a
 * dispatcher thread.  ccq_server_submit may be called from any host thread;
 * queries are admitted in arrival order while their workspace fits the
 * arena and fewer than max_inflight are admitted or running.  Whenever one of
 * the n_streams launch streams is idle, the dispatcher launches everything
 * admitted so far on it -- as one batch (batching = 1, as ccq_batch_execute)
 * or as one ccq_execute per query (batching = 0) -- so queries that arrive
 * while others run join the next launch and overlap with them on the device.
 * Each query's answer is exactly what ccq_execute gives.  A query whose
 * workspace alone exceeds the arena completes with CCQ_E_BUDGET.  The plan
 * and the result buffers of a submitted query must stay alive until its
 * completion has been polled. */
typedef struct ccq_server ccq_server;

typedef struct {
    int64_t hbm_budget_bytes;  /* device arena for workspaces and launch descriptors */
    int32_t max_inflight;      /* queries admitted or running at once (slots) */
    int32_t max_batch;         /* queries per launch (0: max_inflight) */
    int32_t n_streams;         /* launch streams (0: 2) */
    int32_t batching;          /* 1: one batched launch per dispatch; 0: one ccq_execute per query */
    int32_t tiles_per_item;    /* largest batch work item in 2048-row tiles (0: 64); a dispatch with
                                  few tiles in all uses smaller items so they spread over the GPU */
    int32_t no_graphs;         /* 0: each batched dispatch replays a hipGraph captured once per launch
                                  shape (kernel instances, grids, LDS, query count rounded up to a
                                  power of two), its per-query descriptors copied to device memory
                                  first; 1: launch every dispatch directly */
} ccq_server_config;

typedef struct {
    uint64_t ticket;
    int32_t status;            /* CCQ_OK, CCQ_E_BUDGET, or CCQ_E_HIP */
    int32_t pad_;
    double t_submit;           /* host steady clock, seconds (ccq_now) */
    double t_start;            /* when its launch was enqueued (rejected: when rejected) */
    double t_done;             /* when the dispatcher saw its launch finish */
} ccq_completion;

/* Host steady clock in seconds (the clock of ccq_completion). */
double ccq_now(void);

ccq_status ccq_server_create(ccq_context* ctx, const ccq_server_config* cfg, ccq_server** out);
ccq_status ccq_server_submit(ccq_server* s, const ccq_plan* p, const ccq_result* r, uint64_t* ticket);
/* Move up to max completions into out (oldest first); *n = how many. */
ccq_status ccq_server_poll(ccq_server* s, ccq_completion* out, int32_t max, int32_t* n);
/* Wait until every submitted query has completed (CCQ_E_BUSY on timeout). */
ccq_status ccq_server_drain(ccq_server* s, double timeout_s);
/* Finishes outstanding queries, then stops the dispatcher and frees the arena. */
void ccq_server_destroy(ccq_server* s);

#ifdef __cplusplus
}
#endif

#endif /* CCQ_H */

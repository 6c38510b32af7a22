/*
 * colmerge.h -- C ABI of the MI355X (gfx950) column-merge library.
 *
 * The operation is the online merge of one dictionary-encoded column of a
 * read-optimized column store (Krueger et al., "Fast Updates on
 * Read-Optimized Databases Using Multi-Core CPUs", arXiv 1109.6885):
 *
 *   inputs   U_M  sorted unique main dictionary            (Section 3)
 *            M    main codes, bit-packed at width E_C = w  (Section 4.1)
 *            D    delta values in append order             (Section 3)
 *   outputs  U'   sorted unique merged dictionary          (Eq. 3)
 *            M'   N_M + N_D codes at width E_C' = w'       (Eqs. 2, 4)
 *            X_M, X_D translation tables (old -> new code) (Section 5.3)
 *
 * Step 1(a) builds the delta dictionary U_D and the index of every delta
 * row in it, Step 1(b) merges U_M and U_D into U' while emitting X_M and
 * X_D, Step 2(a) computes w' (Eq. 4) and Step 2(b) rewrites every main code
 * through X_M and appends the delta codes through X_D (Eq. 11).
 *
 * Conventions (the paper leaves them open):
 *  - Value types: MC_U32 (4 bytes) and MC_U64 (8 bytes) are unsigned
 *    little-endian integers in numeric order; MC_STR16 is 16 raw bytes
 *    ordered as unsigned bytes, first byte most significant (memcmp).
 *  - Packed codes: code i occupies stream bits [i*w, (i+1)*w), least
 *    significant bit first; stream bit b is bit (b % 64) of 64-bit word
 *    b / 64.  Result bits beyond N'*w' in the last word are zero.
 *  - width(n) = ceil(log2 n) for n >= 2, and 1 for n <= 1.
 *  - Every U_M entry is kept (Eq. 3 unions with U_M) and every row is kept
 *    (insert-only updates, Eq. 2).
 *
 * Memory: every data pointer in mc_column_in / mc_column_out and every
 * scratch pointer is a DEVICE pointer owned by the caller.  Value arrays,
 * code arrays and scratch must be 16-byte aligned.  Main code buffers are
 * read only up to word ceil(N_M * w / 64); result code buffers are written
 * up to the capacity returned by mc_merge_bounds (words past W' may be
 * overwritten with zeros).  The library never allocates or frees caller
 * memory and never synchronizes the caller's stream: every mc_merge_* call
 * only enqueues work on `stream` and returns; results are valid once the
 * stream reaches that point.
 *
 * Errors: every call returns MC_OK (0) or a negative mc_status.  A failed
 * call enqueues nothing and leaves the inputs untouched.  Data errors that
 * only the device can see (a main code >= |U_M|, a delta index out of range)
 * are reported in mc_result.error after the stream completes; the outputs
 * are then unspecified but every access stays inside the buffers.
 * mc_last_error() returns a message for the calling thread's last failure.
 *
 * Threading: an mc_ctx is used from one host thread at a time.  Different
 * contexts, or one context on different streams with different scratch
 * buffers, may run concurrently.  One kernel of a single-column merge (the
 * full sort that Step 1(a) falls back on when values share long prefixes)
 * needs all of its workgroups resident at once; it launches at most one per
 * two compute units, so six such merges can run it side by side (HIP runs
 * at most 4 kernels at a time with its default of 4 hardware queues).  Should
 * more ever compete, its bounded waits end with MC_DEVERR_SPIN in
 * mc_result.error instead of hanging.
 */
#ifndef COLMERGE_H
#define COLMERGE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

struct ihipStream_t; /* hipStream_t is `struct ihipStream_t *` */

typedef struct mc_ctx mc_ctx;
typedef struct mc_graph mc_graph;

typedef enum mc_type { MC_U32 = 0, MC_U64 = 1, MC_STR16 = 2 } mc_type;

typedef enum mc_status {
    MC_OK = 0,
    MC_E_ARG = -1,   /* null pointer, size or width out of range, misaligned */
    MC_E_CAP = -2,   /* an output or scratch capacity is below the bounds    */
    MC_E_NOMEM = -3, /* host-side allocation failed                           */
    MC_E_HIP = -4,   /* a HIP runtime call failed (see mc_last_error)         */
    MC_E_DATA = -5   /* invalid data found by the device (validate mode)      */
} mc_status;

/* Bits of mc_result.error. */
#define MC_DEVERR_CODE_RANGE 1u  /* a main code >= |U_M| was read            */
#define MC_DEVERR_DELTA_RANGE 2u /* a delta index >= |U_D| (internal)        */
#define MC_DEVERR_SPIN 4u        /* a cross-workgroup wait hit its bound     */
#define MC_DEVERR_ORDER 8u       /* a dictionary is not strictly increasing  */
/* Outside validate mode (mc_ctx_set_validate) the device does not check the
 * order of U_M (a full check costs a pass over it); a U_M out of order gives
 * an undefined result, and where a merge tile meets the inconsistency it
 * stays empty and sets MC_DEVERR_ORDER instead of reading past its inputs. */

/* Result scalars, written by the device (caller-allocated device memory). */
typedef struct mc_result {
    uint64_t new_dict_len;    /* |U'|                                        */
    uint64_t new_codes_words; /* W' = ceil((N_M + N_D) * w' / 64)            */
    uint64_t delta_dict_len;  /* |U_D|                                       */
    uint32_t new_bitwidth;    /* w' (Eq. 4)                                  */
    uint32_t error;           /* MC_DEVERR_* bits, 0 if none                 */
} mc_result;

/* One column's inputs (device pointers). */
typedef struct mc_column_in {
    int32_t type;              /* mc_type                                    */
    uint32_t bitwidth;         /* w, 1..32, with |U_M| <= 2^w                */
    const void *main_dict;     /* U_M: main_dict_len values, strictly increasing */
    uint64_t main_dict_len;    /* |U_M|; 0 only if main_rows == 0            */
    const uint64_t *main_codes;/* packed main codes, ceil(main_rows*w/64) words */
    uint64_t main_rows;        /* N_M                                        */
    const void *delta_values;  /* D: delta_rows values in append order       */
    uint64_t delta_rows;       /* N_D, < 2^30                                */
} mc_column_in;

/* One column's outputs (device pointers, caller-allocated). */
typedef struct mc_column_out {
    void *new_dict;               /* U': capacity new_dict_cap values        */
    uint64_t new_dict_cap;        /* >= dict_cap of mc_merge_bounds          */
    uint64_t *new_codes;          /* M': capacity new_codes_cap_words words  */
    uint64_t new_codes_cap_words; /* >= codes_words of mc_merge_bounds       */
    uint32_t *x_main;             /* X_M (|U_M| entries) or NULL             */
    uint32_t *x_delta;            /* X_D (delta_rows entries) or NULL        */
    mc_result *result;            /* device scalars, required                */
} mc_column_out;

/* ---- contexts -------------------------------------------------------- */

/* Create a context bound to HIP device `device`. */
int mc_ctx_create(int device, mc_ctx **out);
void mc_ctx_destroy(mc_ctx *ctx);

/* Message for the calling thread's last failed call ("" if none). */
const char *mc_last_error(void);

/* Validate mode (off by default).  The paper's main dictionary is sorted and
 * free of duplicates and every main code indexes it (Sections 3 and 4.1);
 * the merge relies on both.  With validate mode on, mc_merge_column,
 * mc_merge_column_naive, mc_merge_column_indexed and
 * mc_merge_columns_batched become synchronous checkers:
 *  1. a device pass checks that every U_M is strictly increasing and the
 *     call waits for it; a dictionary out of order returns MC_E_DATA (the
 *     result's error word holds MC_DEVERR_ORDER; nothing else is written);
 *  2. the merge is enqueued as usual, the call waits for the stream, and
 *     returns MC_E_DATA if the device found a main code >= |U_M|
 *     (MC_DEVERR_CODE_RANGE) or any other data error bit.
 * mc_last_error names the column and the bit.  Validate mode must not be on
 * while the stream is being captured into a graph (the call waits on it);
 * a batched call that captures a graph (graph != NULL) validates before the
 * capture and waits after the launch. */
int mc_ctx_set_validate(mc_ctx *ctx, int enable);

/* ---- sizing (host only, no device access) ---------------------------- */

/* Worst-case sizes for one column, from the input sizes alone:
 *   dict_cap      = |U_M| + N_D values for U'
 *   codes_words   = ceil((N_M + N_D) * width(|U_M| + N_D) / 64) rounded up
 *                   to a multiple of 2 (room for 128-bit stores)
 *   scratch_bytes = device workspace for mc_merge_column.
 * These bounds need no device read, so they serve admission control and
 * graph capture (outputs sized before the real |U'| is known). */
int mc_merge_bounds(const mc_column_in *in, uint64_t *dict_cap,
                    uint64_t *codes_words, uint64_t *scratch_bytes);
/* The same for merges on `ctx` (its tuning can route a delta to the
 * hashing route of Step 1(a), which needs more scratch; NULL: defaults). */
int mc_merge_bounds_ctx(const mc_ctx *ctx, const mc_column_in *in,
                        uint64_t *dict_cap, uint64_t *codes_words,
                        uint64_t *scratch_bytes);

/* ---- the merge of one column (Section 5, Steps 1(a) to 2(b)) --------- */

/* Enqueue the whole merge of one column on `stream`.  `scratch` is a
 * device workspace of at least scratch_bytes (mc_merge_bounds); its
 * contents need not be initialized.  X_M / X_D are written only if the
 * out pointers are non-NULL. */
int mc_merge_column(mc_ctx *ctx, const mc_column_in *in,
                    const mc_column_out *out, void *scratch,
                    uint64_t scratch_bytes, struct ihipStream_t *stream);

/* The same merge with the unoptimized Step 2(b) of Section 5.2 (cost of
 * Eq. 5): each main row's value is read from U_M and its new code found by
 * binary search in U'; each delta value is searched directly.  Same inputs,
 * outputs, scratch and results as mc_merge_column; it exists to measure the
 * translation tables of Section 5.3 against the route they replace
 * (Section 7.1).  X_M / X_D outputs, if requested, are still written. */
int mc_merge_column_naive(mc_ctx *ctx, const mc_column_in *in,
                          const mc_column_out *out, void *scratch,
                          uint64_t scratch_bytes, struct ihipStream_t *stream);

/* ---- allocation-free merge -------------------------------------------- */

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the merge
 * of mc_merge_column (same kernels, same results, same outputs) with its
 * workspace in a device array of MC_NOALLOC_SCRATCH_BYTES that the library
 * holds on every GPU it runs on, from the first mc_ctx_create on that device
 * until the process ends.  The caller still passes the inputs and outputs.
 * The call allocates nothing: no hipMalloc / hipFree, no allocating library
 * routine, no step-timing events (mc_ctx_set_timing does not apply to it).
 *
 * Limit: a column whose workspace (scratch_bytes of mc_merge_bounds_ctx on
 * ctx) exceeds MC_NOALLOC_SCRATCH_BYTES is rejected with MC_E_CAP before
 * anything is enqueued; 64 MiB holds, e.g., a 1M-row u64 delta against a
 * 1M-entry dictionary.  Every call on one GPU shares that GPU's array (the
 * part that must start at zero is cleared by each call on its stream), so
 * calls whose work overlaps on one GPU -- different streams, or different
 * host threads -- race; serialize them on one stream. */
#define MC_NOALLOC_SCRATCH_BYTES (64ull << 20)
int mc_merge_column_noalloc(mc_ctx *ctx, const mc_column_in *in,
                            const mc_column_out *out,
                            struct ihipStream_t *stream);

/* ---- single steps (the same kernels as mc_merge_column) --------------- */

/* Step 1(a), modified form (Sections 5.1 and 5.3): sorted unique delta
 * dictionary u_d (delta_rows capacity, same value type) and each delta
 * row's index in it (drank, delta_rows entries).  *d_count (device u64)
 * receives |U_D|.  Scratch: mc_delta_dictionary_scratch bytes (enough
 * for either route of Step 1(a), whatever the context's tuning). */
int mc_delta_dictionary(mc_ctx *ctx, int32_t type, const void *delta_values,
                        uint64_t delta_rows, void *u_d, uint32_t *drank,
                        uint64_t *d_count, void *scratch,
                        uint64_t scratch_bytes, struct ihipStream_t *stream);
int mc_delta_dictionary_scratch(int32_t type, uint64_t delta_rows,
                                uint64_t *scratch_bytes);

/* Step 1(b) and Step 2(a) (Sections 5.1, 5.3, 6.2.1; Eq. 4): merge the
 * sorted unique dictionaries u_m (n_um values) and u_d (*d_n_ud values,
 * read on the device, at most n_ud_max) into u_new with tables x_m and x_d.
 * Writes result->new_dict_len, ->new_bitwidth and ->new_codes_words for a
 * merged column of `rows_total` rows.  Scratch: mc_merge_dictionaries_scratch. */
int mc_merge_dictionaries(mc_ctx *ctx, int32_t type, const void *u_m,
                          uint64_t n_um, const void *u_d,
                          const uint64_t *d_n_ud, uint64_t n_ud_max,
                          void *u_new, uint32_t *x_m, uint32_t *x_d,
                          uint64_t rows_total, mc_result *result,
                          void *scratch, uint64_t scratch_bytes,
                          struct ihipStream_t *stream);
int mc_merge_dictionaries_scratch(uint64_t n_um, uint64_t n_ud_max,
                                  uint64_t *scratch_bytes);

/* Step 2(b), modified form (Eq. 11; Section 6.2.2): out[i] = x_m[main[i]]
 * for i < n_main, out[n_main + j] = x_d[drank[j]] for j < n_delta, packed
 * at width result->new_bitwidth (read on the device).  x_m has n_um
 * entries, x_d has result->delta_dict_len entries.  Writes
 * ceil((n_main + n_delta) * w' / 64) words (rounded up to even, zero
 * padded) into out (capacity out_cap_words). */
int mc_reencode(mc_ctx *ctx, const uint64_t *main_codes, uint64_t n_main,
                uint32_t w, const uint32_t *x_m, uint64_t n_um,
                const uint32_t *drank, uint64_t n_delta, const uint32_t *x_d,
                mc_result *result, uint64_t *out, uint64_t out_cap_words,
                struct ihipStream_t *stream);

/* ---- delta index: Step 1(a)'s hashing done as rows are appended ------- */

/* The paper keeps a CSB+ tree beside each delta partition so that Step 1(a)
 * is a walk over its leaves and the insert cost is paid per update (Section
 * 4, Section 6.1; other delta structures are its stated future work).  A
 * delta index does the same job with the hashing route of Step 1(a): each
 * appended batch of rows is hashed into an open-addressing table of
 * representative rows, and the batch's new distinct values are added to a
 * distinct list, so that a merge (mc_merge_column_indexed) starts from the
 * distinct values and skips the hashing; T_U of Eq. 1 then carries it.
 *
 * workspace:  device memory of mc_delta_index_bytes (16-byte aligned),
 *             owned by the caller; reset it before the first append and
 *             after each merge that consumed the delta;
 * capacity:   delta rows it can index (< 2^30);
 * type:       mc_type of the delta values. */
typedef struct mc_delta_index {
    void *workspace;
    uint64_t workspace_bytes;
    uint64_t capacity;
    int32_t type;
    uint32_t reserved; /* zero */
} mc_delta_index;

int mc_delta_index_bytes(int32_t type, uint64_t capacity, uint64_t *bytes);
/* Empty the index (stream-ordered). */
int mc_delta_index_reset(mc_ctx *ctx, const mc_delta_index *index,
                         struct ihipStream_t *stream);
/* Index rows [row0, row0 + rows) of the delta (device values, all rows
 * before row0 already indexed, each row exactly once, in order;
 * row0 + rows <= capacity).  Stream-ordered. */
int mc_delta_index_append(mc_ctx *ctx, const mc_delta_index *index,
                          const void *delta_values, uint64_t row0, uint64_t rows,
                          struct ihipStream_t *stream);
/* The merge of mc_merge_column with Step 1(a) starting from the index:
 * in->delta_values / delta_rows are the indexed rows [0, delta_rows), in
 * the same buffer that was indexed.  Same outputs and error word (plus the
 * index's own error bits).  Scratch: mc_merge_indexed_bounds bytes. */
int mc_merge_indexed_bounds(const mc_column_in *in, uint64_t *scratch_bytes);
int mc_merge_column_indexed(mc_ctx *ctx, const mc_column_in *in,
                            const mc_delta_index *index,
                            const mc_column_out *out, void *scratch,
                            uint64_t scratch_bytes, struct ihipStream_t *stream);

/* ---- many columns at once (Section 6.2.1, scheme (i)) ----------------- */

/* Worst-case scratch for merging ncols columns in one batched call on a
 * context with the default tuning.  Every column takes the Step 1(a) route
 * it would take alone (deltas of 2^21 rows or more hash first), so columns
 * on the hashing route need its table and distinct-value buffers too. */
int mc_merge_batched_bounds(const mc_column_in *ins, uint32_t ncols,
                            uint64_t *scratch_bytes);
/* The same for batched merges on `ctx`, whose hash_min_rows can send more
 * deltas to the hashing route (NULL: defaults). */
int mc_merge_batched_bounds_ctx(const mc_ctx *ctx, const mc_column_in *ins,
                                uint32_t ncols, uint64_t *scratch_bytes);

/* Enqueue the merge of ncols independent columns (uneven sizes and value
 * types).  Two forms, chosen by the context's tuning (batched_launch):
 *  MC_BATCHED_PHASES      one launch per phase, each covering the tiles of
 *                         all columns (about 70 launches whatever ncols);
 *  MC_BATCHED_PERSISTENT  (disabled: mc_ctx_set_tuning refuses it with
 *                         MC_E_ARG; its launch stalled on the GPU, also
 *                         with one workgroup, and the cause is not found)
 *                         one persistent launch (after a small clearing
 *                         kernel): its workgroups take work items -- a tile
 *                         or a slice of one step of one column -- from one
 *                         device counter, in an order where every item's
 *                         inputs come from items taken before it, so a
 *                         workgroup only ever waits for items that running
 *                         workgroups hold (Section 6.2.1, scheme (i), a
 *                         task queue).  Columns overlap: one column's merge
 *                         runs beside another's sort.  Every wait is bounded
 *                         and reports MC_DEVERR_SPIN in the column's error
 *                         word if it ever overruns.
 * Both give the same results.  If `graph`
 * is non-NULL the sequence is captured once into a HIP graph (returned in
 * *graph, reusable with mc_graph_launch for the same buffers) and launched;
 * otherwise it is enqueued directly.  ins/outs are host arrays of ncols
 * descriptors whose pointers are device pointers. */
int mc_merge_columns_batched(mc_ctx *ctx, const mc_column_in *ins,
                             const mc_column_out *outs, uint32_t ncols,
                             void *scratch, uint64_t scratch_bytes,
                             struct ihipStream_t *stream, mc_graph **graph);
int mc_graph_launch(mc_graph *graph, struct ihipStream_t *stream);
void mc_graph_destroy(mc_graph *graph);

/* ---- tuning ------------------------------------------------------------ */

/* Launch shapes a context uses for every later merge (single column and
 * batched; a captured graph keeps the shapes it was captured with).
 *   repack_codes: rows per Step 2(b) workgroup tile, 1024, 2048 (default)
 *                 or 4096, i.e. 4, 8 or 16 codes per thread;
 *   prefix_run:   values per run of equal prefix that Step 1(a) aims for
 *                 when it picks how many leading digits to sort globally
 *                 (4 .. 1024, default 32; more runs -> more radix passes,
 *                 longer runs -> more work in the LDS windows);
 *   hash_min_rows: deltas of at least this many rows deduplicate by hashing
 *                 before sorting (0: the default, 2^21; 1: always);
 *   batched_launch: MC_BATCHED_PHASES (0, default); MC_BATCHED_PERSISTENT
 *                 is refused for now (see mc_merge_columns_batched);
 *   persist_workers: workgroups of the persistent launch (0: as many as the
 *                 GPU holds at once; any count >= 1 completes);
 *   persist_repack: Step 2(b) tiles per work item of the persistent launch
 *                 (0: default 4; at most 1024);
 *   persist_merge: dictionary-merge tiles per work item (0: default 2; at
 *                 most 1024);
 *   hash_dict_ratio: a delta of at least 4096 rows also hashes first when
 *                 it has at least this many times as many rows as U_M has
 *                 entries (0: the default, 64; 0xFFFFFFFF: never): most
 *                 of its rows then repeat a few values, whose runs of equal
 *                 prefix the prefix sort cannot order in place.
 * The results do not depend on them. */
#define MC_BATCHED_PHASES 0u
#define MC_BATCHED_PERSISTENT 1u
typedef struct mc_tuning {
    uint32_t repack_codes;
    uint32_t prefix_run;
    uint32_t hash_min_rows;
    uint32_t batched_launch;
    uint32_t persist_workers;
    uint32_t persist_repack;
    uint32_t persist_merge;
    uint32_t hash_dict_ratio;
} mc_tuning;

/* MC_E_ARG if a value is outside the ranges above (the context keeps its
 * previous shapes). */
int mc_ctx_set_tuning(mc_ctx *ctx, const mc_tuning *tuning);
int mc_ctx_get_tuning(const mc_ctx *ctx, mc_tuning *tuning);

/* Autotuner for the batched merge: runs the given batch (same arguments as
 * mc_merge_columns_batched, no graph) with each candidate shape -- first
 * repack_codes in {1024, 2048, 4096}, then, with the best of those,
 * prefix_run in {16, 32, 64} -- timing each with HIP events on `stream`
 * (best of two runs after one warm-up run), stores the fastest in the
 * context and returns it in *chosen.  times_ms (nullable) receives the 6
 * candidate times in that order.  It synchronizes the stream; the outputs
 * hold the batch's merge result afterwards. */
int mc_autotune_batched(mc_ctx *ctx, const mc_column_in *ins,
                        const mc_column_out *outs, uint32_t ncols,
                        void *scratch, uint64_t scratch_bytes,
                        struct ihipStream_t *stream, mc_tuning *chosen,
                        float *times_ms);

/* ---- launch shapes per column class ------------------------------------ */

/* Columns of a batch fall into tuning classes by value type, input code
 * width (1-8, 9-16, 17-24, 25-32 bits) and size (main + delta rows below
 * 2^21, below 2^24, or more): class = (type * 4 + width class) * 3 + size
 * class, 3 x 4 x 3 = MC_TUNE_CLASSES classes.  A context caches shapes per
 * class; in a batched merge a column of a class with cached shapes uses
 * their repack_codes and prefix_run (one re-encode launch per tile size in
 * use), every other column the context's tuning.  The persistent batched
 * launch, with one tile size, ignores the cache. */
#define MC_TUNE_CLASSES 36u

/* *cls = the class of column `in`.  MC_E_ARG for a null argument or a
 * column descriptor that mc_merge_column would refuse. */
int mc_tune_class(const mc_column_in *in, uint32_t *cls);

/* Cache the shapes of class `cls` (< MC_TUNE_CLASSES); tuning null removes
 * them.  MC_E_ARG for a null context, a class out of range, or
 * repack_codes / prefix_run outside the ranges of mc_tuning. */
int mc_ctx_set_class_tuning(mc_ctx *ctx, uint32_t cls, const mc_tuning *tuning);

/* The shapes a column of class `cls` gets: the context's tuning with the
 * class's cached repack_codes and prefix_run, if any (*is_set, nullable, is
 * 1 then, else 0). */
int mc_ctx_get_class_tuning(const mc_ctx *ctx, uint32_t cls, mc_tuning *tuning,
                            int *is_set);

/* Autotuner per class: for every class present in the batch (arguments as
 * for mc_merge_columns_batched, no graph), runs the batch's columns of that
 * class alone with each candidate shape -- repack_codes in {1024, 2048,
 * 4096}, then prefix_run in {16, 32, 64} with the best of those -- timing
 * each with HIP events on `stream` (best of three runs after one warm-up
 * run), and caches the fastest for the class in the context.  *classes
 * (nullable) receives the number of classes tuned.  It synchronizes the
 * stream; the outputs hold the batch's merge result afterwards. */
int mc_autotune_batched_classes(mc_ctx *ctx, const mc_column_in *ins,
                                const mc_column_out *outs, uint32_t ncols,
                                void *scratch, uint64_t scratch_bytes,
                                struct ihipStream_t *stream, uint32_t *classes);

/* ---- step timing (for measurement) ------------------------------------ */

/* Enabling (or re-enabling) timing starts a new measurement: from then on
 * every mc_merge_column call records HIP events around each step on its
 * own stream.  mc_ctx_step_times waits for the last recorded merge and
 * writes the AVERAGE milliseconds over the recorded merges of the first n
 * (<= MC_STEP_TIMES) of:
 * [0] workspace clear + delta sort, [1] delta dictionary emit,
 * [2] dictionary merge and width, [3] re-encode (X_M compaction and the
 * re-encode kernel), [4] whole call, [5] the re-encode kernel alone. */
#define MC_STEP_TIMES 6
int mc_ctx_set_timing(mc_ctx *ctx, int enable);
int mc_ctx_step_times(mc_ctx *ctx, float *ms, uint32_t n);

/* ---- measurement ------------------------------------------------------- */

/* Copy `bytes` (a multiple of 16; 16-byte aligned device buffers) with a
 * plain 128-bit streaming kernel.  Not part of the merge: it measures the
 * achievable HBM bandwidth beside the merge kernels and serves as the
 * known-traffic kernel that calibrates hardware byte counters. */
int mc_copy_bytes(mc_ctx *ctx, const void *src, void *dst, uint64_t bytes,
                  struct ihipStream_t *stream);

/* Random-gather reference: out[i] = table[idx[i] % n_table] for i < n,
 * with 2- or 4-byte table entries (device buffers; idx and out hold n
 * entries).  Not part of the merge: it measures how fast random lookups
 * into a table of a given footprint run, which bounds the translation-table
 * lookups of Step 2(b) (Eq. 11), beside the streaming bound of
 * mc_copy_bytes. */
int mc_gather_ref(mc_ctx *ctx, const uint32_t *idx, uint64_t n,
                  const void *table, uint32_t entry_bytes, uint32_t n_table,
                  uint32_t *out, struct ihipStream_t *stream);

#ifdef __cplusplus
}
#endif
#endif /* COLMERGE_H */
